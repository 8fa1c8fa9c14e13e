// rwpt_pairstep.h -- per-candidate steps of the row-broadcast pair kernels
// (internal to the HIP code).
//
// In the row-broadcast tiling a 16-lane row of a wave holds 16 particles i of
// a tile, and every lane of the row has loaded one candidate j.  Step K
// broadcasts lane K's candidate to the whole row (a DPP row_share, which the
// compiler folds into the consuming subtract) and every lane evaluates the
// pair (i, j_K).  A chunk is the 16 steps K = 0..15.
//
// The row-sum and exchange kernels and the instruction-rate probe all call the
// chunk functions below, so the probe times exactly the kernels' sequence.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

namespace rwpt {

// Co-location weight exp(-s2 / sigma^2) (Eq. 3 without prefactor): binary32
// uses the hardware exp2 with the scale -log2(e)/sigma^2; binary64 uses the
// library exp.
__device__ __forceinline__ float kweight(float s2, float escale) {
  return __builtin_amdgcn_exp2f(s2 * escale);
}
__device__ __forceinline__ double kweight(double s2, double escale) { return exp(s2 * escale); }

// Value of lane K of this lane's 16-lane row (DPP row_share).
template <int K>
__device__ __forceinline__ float rshare(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + K, 0xf,
                                                               0xf, false));
}

// Compile-time loop K = Begin..End-1 (each step needs K as a constant).
template <int K, int N>
struct Steps {
  template <typename F>
  __device__ __forceinline__ static void run(F&& f) {
    f(std::integral_constant<int, K>{});
    Steps<K + 1, N>::run(f);
  }
};
template <int N>
struct Steps<N, N> {
  template <typename F>
  __device__ __forceinline__ static void run(F&&) {}
};

// Weight of the pair (this lane's particle, candidate K of the row), zero
// unless the lane is active and s^2 <= rc2 (the cutoff predicate of the
// neighbour search).  s^2 = fma(d2, d2, fma(d1, d1, d0 * d0)).
template <int K, int DIM>
__device__ __forceinline__ float row_weight(const float (&xj)[DIM], const float (&xi)[DIM], float rc2, float esc,
                                            bool act) {
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
  const float w = kweight(s2, esc);
  return (act && s2 <= rc2) ? w : 0.0f;
}

// Row sum over one chunk: sum over K of w(i, j_K).
template <int DIM>
__device__ __forceinline__ float rowsum_chunk(const float (&xj)[DIM], const float (&xi)[DIM], float rc2, float esc,
                                              bool act) {
  float a = 0.0f;
  Steps<0, 16>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    a += row_weight<K, DIM>(xj, xi, rc2, esc, act);
  });
  return a;
}

// Exchange over one chunk, symmetric normalisation: accr[s] += w (q_j + q_i)
// (m_j[s] - M_i[s]) with q = 1 / r, i.e. twice the symmetric P_ij times the
// mass difference.
template <int DIM, int SMAX>
__device__ __forceinline__ void exchange_chunk_sym(const float (&xj)[DIM], const float (&xi)[DIM], float qj, float qi,
                                                   const float (&mj)[SMAX], const float (&Mi)[SMAX], float rc2,
                                                   float esc, bool act, float (&accr)[SMAX]) {
  Steps<0, 16>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const float w = row_weight<K, DIM>(xj, xi, rc2, esc, act);
    const float p = w * (rshare<K>(qj) + qi);  // 2 * symmetric P_ij
#pragma unroll
    for (int s = 0; s < SMAX; ++s) accr[s] += p * (rshare<K>(mj[s]) - Mi[s]);
  });
}

// Exchange over one chunk, row normalisation: rr += w and accr[s] += w
// (m_j[s] - M_i[s]); the caller divides by r_i = rr summed over all chunks.
template <int DIM, int SMAX>
__device__ __forceinline__ void exchange_chunk_row(const float (&xj)[DIM], const float (&xi)[DIM],
                                                   const float (&mj)[SMAX], const float (&Mi)[SMAX], float rc2,
                                                   float esc, bool act, float& rr, float (&accr)[SMAX]) {
  Steps<0, 16>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const float w = row_weight<K, DIM>(xj, xi, rc2, esc, act);
    rr += w;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) accr[s] += w * (rshare<K>(mj[s]) - Mi[s]);
  });
}

}  // namespace rwpt
