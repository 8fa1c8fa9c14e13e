// rwpt_probe.hip -- register-only kernels that measure the instruction rates
// the row-broadcast pair kernels can reach on this device.
//
// The pair kernels are bound by their VALU instruction stream (one exp, the
// distance, the cutoff predicate and the mass products per candidate), so a
// published FLOP/s peak says little about how close they run to what the
// hardware can do.  These kernels run the same per-candidate code
// (rowsum_chunk / exchange_chunk_sym of rwpt_pairstep.h) on operands held in
// registers -- no loads, no cursor, no tile bookkeeping -- at full occupancy,
// which gives the attainable candidate-evaluation rate of each kernel's inner
// loop.  Two more kernels give the plain binary32 FMA and exp2 issue rates.
#include <hip/hip_runtime.h>

#include "rwpt_kernels.h"
#include "rwpt_pairstep.h"

namespace rwpt {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kUnrollP = 16;  // operations per chain per iteration

// Makes v opaque to the optimiser (it may have changed) without emitting code,
// so the chunk is recomputed every iteration as if its operands were loaded.
__device__ __forceinline__ void opaque(float& v) { asm volatile("" : "+v"(v)); }

__global__ __launch_bounds__(kProbeBlock) void k_probe_fma(float* __restrict__ out, int iters, float b) {
  float a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = 1e-3f * (float)threadIdx.x + (float)k;
  const float c = 1.0f - b;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kUnrollP; ++r) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) a[k] = __builtin_fmaf(a[k], b, c);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_exp(float* __restrict__ out, int iters) {
  float e[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) e[k] = 1e-4f * (float)threadIdx.x + 0.1f * (float)k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kUnrollP; ++r) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) e[k] = __builtin_amdgcn_exp2f(-e[k]);  // stays in [0.5, 1]
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += e[k];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

// Particle and candidate coordinates on a lattice of spacing h/8 in [0, 2h),
// so that with h near the cutoff some pairs fall inside it and some outside.
template <int DIM>
__device__ __forceinline__ void probe_coords(int lane, float h, float (&xi)[DIM], float (&xj)[DIM]) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    xi[k] = 0.125f * h * (float)((lane * (3 + 2 * k)) & 15);
    xj[k] = 0.125f * h * (float)((lane * (5 + 2 * k) + 7) & 15);
  }
}

template <int DIM>
__global__ __launch_bounds__(kProbeBlock) void k_probe_rowsum(float* __restrict__ out, int chunks, float rc2,
                                                              float esc, float h) {
  const int lane = threadIdx.x & 63;
  float xi[DIM], xj[DIM];
  probe_coords<DIM>(lane, h, xi, xj);
  const bool act = lane < 64 + chunks;  // true, but not known to the compiler
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) opaque(xj[k]);
    acc += (double)rowsum_chunk<DIM>(xj, xi, rc2, esc, act);
  }
  out[blockIdx.x * kProbeBlock + threadIdx.x] = (float)acc;
}

template <int DIM, int SMAX>
__global__ __launch_bounds__(kProbeBlock) void k_probe_exchange(float* __restrict__ out, int chunks, float rc2,
                                                                float esc, float h) {
  const int lane = threadIdx.x & 63;
  float xi[DIM], xj[DIM], mj[SMAX], Mi[SMAX];
  probe_coords<DIM>(lane, h, xi, xj);
  float qj = 1.0f + 1e-3f * (float)lane;
  const float qi = 1.0f - 1e-3f * (float)lane;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    mj[s] = 1.0f + 0.01f * (float)((lane + s) & 7);
    Mi[s] = 1.0f + 0.01f * (float)((lane * 3 + s) & 7);
  }
  const bool act = lane < 64 + chunks;
  double acc[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) acc[s] = 0.0;
  for (int c = 0; c < chunks; ++c) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) opaque(xj[k]);
    opaque(qj);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) opaque(mj[s]);
    float accr[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) accr[s] = 0.0f;
    exchange_chunk_sym<DIM, SMAX>(xj, xi, qj, qi, mj, Mi, rc2, esc, act, accr);
#pragma unroll
    for (int s = 0; s < SMAX; ++s) acc[s] += (double)accr[s];
  }
  double t = 0.0;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) t += acc[s];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = (float)t;
}

template <int DIM>
hipError_t launch_probe_dim(int kind, int slots, int blocks, int reps, float rc2, float esc, float h, float* out,
                            hipStream_t s) {
  const dim3 g(blocks), b(kProbeBlock);
  if (kind == PROBE_ROWSUM) {
    hipLaunchKernelGGL((k_probe_rowsum<DIM>), g, b, 0, s, out, reps, rc2, esc, h);
  } else if (slots <= 2) {
    hipLaunchKernelGGL((k_probe_exchange<DIM, 2>), g, b, 0, s, out, reps, rc2, esc, h);
  } else if (slots <= 4) {
    hipLaunchKernelGGL((k_probe_exchange<DIM, 4>), g, b, 0, s, out, reps, rc2, esc, h);
  } else {
    hipLaunchKernelGGL((k_probe_exchange<DIM, 8>), g, b, 0, s, out, reps, rc2, esc, h);
  }
  return hipGetLastError();
}

}  // namespace

int probe_block() { return kProbeBlock; }

int64_t probe_ops_per_lane(int kind, int reps) {
  if (kind == PROBE_FMA || kind == PROBE_EXP) return (int64_t)reps * kChains * kUnrollP;
  return (int64_t)reps * 16;  // candidate evaluations: 16 per chunk
}

hipError_t launch_probe(int kind, int dim, int slots, int blocks, int reps, float rc2, float esc, float h, float* out,
                        hipStream_t s) {
  if (kind == PROBE_FMA) {
    hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(kProbeBlock), 0, s, out, reps, 0.5f);
    return hipGetLastError();
  }
  if (kind == PROBE_EXP) {
    hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(kProbeBlock), 0, s, out, reps);
    return hipGetLastError();
  }
  if (dim == 1) return launch_probe_dim<1>(kind, slots, blocks, reps, rc2, esc, h, out, s);
  if (dim == 2) return launch_probe_dim<2>(kind, slots, blocks, reps, rc2, esc, h, out, s);
  return launch_probe_dim<3>(kind, slots, blocks, reps, rc2, esc, h, out, s);
}

}  // namespace rwpt
