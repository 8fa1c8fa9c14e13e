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
// library exp (the table form exp_tab below is what the binary64 kernels use).
__device__ __forceinline__ float kweight(float s2, float escale) {
  return __builtin_amdgcn_exp2f(s2 * escale);
}
__device__ __forceinline__ double kweight(double s2, double escale) { return exp(s2 * escale); }

// 2^(j/64), j = 0..63, each correctly rounded to binary64.
__device__ constexpr double kExp2Frac[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

// Binary64 exp(x) for x <= 0 (table-driven): x = (64 n + j) ln2/64 + r with
// |r| <= ln2/128, the product t ln2/64 subtracted in two parts (a 32-bit head,
// exact for |t| < 2^21, and the tail); then exp(x) = 2^n 2^(j/64) (1 + q) with
// q = e^r - 1 = r (1 + r/2 + r^2/6 + r^3/24 + r^4/120), whose truncation is
// below 2^-54 relative.  Within 1.1 ulp of exp on [-745, 0]; arguments below
// -1000 return 0.  tbl holds kExp2Frac.
__device__ __forceinline__ double exp_tab(double x, const double* __restrict__ tbl) {
  constexpr double kInvLn2_64 = 0x1.71547652b82fep+6;   // 64 / ln 2
  constexpr double kLn2_64Hi = 0x1.62e42fee00000p-7;    // ln 2 / 64, head
  constexpr double kLn2_64Lo = 0x1.a39ef35793c76p-39;   // ln 2 / 64 - head
  x = __builtin_fmax(x, -1000.0);
  const double t = __builtin_rint(x * kInvLn2_64);
  double r = __builtin_fma(-t, kLn2_64Hi, x);
  r = __builtin_fma(-t, kLn2_64Lo, r);
  const int k = (int)t;
  double p = 1.0 / 120.0;
  p = __builtin_fma(p, r, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  const double q = p * r;
  const double f = tbl[k & 63];
  return __builtin_ldexp(__builtin_fma(f, q, f), k >> 6);
}

// Weight evaluator of the pair kernels.  setup() must be called by every
// thread of the block before any of them returns: the binary64 form fills a
// block-shared copy of kExp2Frac (one barrier); the binary32 form is the
// hardware exp2 and needs nothing.
template <typename T>
struct WeightFn {
  __device__ __forceinline__ void setup() {}
  __device__ __forceinline__ T operator()(T s2, T escale) const { return kweight(s2, escale); }
};
template <>
struct WeightFn<double> {
  const double* tbl;
  __device__ __forceinline__ void setup() {
    __shared__ double sh_tbl[64];
    if (threadIdx.x < 64) sh_tbl[threadIdx.x] = kExp2Frac[threadIdx.x];
    __syncthreads();
    tbl = sh_tbl;
  }
  __device__ __forceinline__ double operator()(double s2, double escale) const {
    return exp_tab(s2 * escale, tbl);
  }
};

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

// Row sum over one chunk: sum over K of w(i, j_K).  NK < 16: only the
// first NK lanes of each row hold candidates (a segment's short last chunk).
template <int DIM, int NK = 16>
__device__ __forceinline__ float rowsum_chunk(const float (&xj)[DIM], const float (&xi)[DIM], float rc2, float esc,
                                              bool act) {
  float a = 0.0f;
  Steps<0, NK>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    a += row_weight<K, DIM>(xj, xi, rc2, esc, act);
  });
  return a;
}

// Exchange over one chunk, symmetric normalisation: accr[s] += w (q_j + q_i)
// (m_j[s] - M_i[s]) with q = 1 / r, i.e. twice the symmetric P_ij times the
// mass difference.
template <int DIM, int SMAX, int NK = 16>
__device__ __forceinline__ void exchange_chunk_sym(const float (&xj)[DIM], const float (&xi)[DIM], float qj, float qi,
                                                   const float (&mj)[SMAX], const float (&Mi)[SMAX], float rc2,
                                                   float esc, bool act, float (&accr)[SMAX]) {
  Steps<0, NK>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const float w = row_weight<K, DIM>(xj, xi, rc2, esc, act);
    const float p = w * (rshare<K>(qj) + qi);  // 2 * symmetric P_ij
#pragma unroll
    for (int s = 0; s < SMAX; ++s) accr[s] += p * (rshare<K>(mj[s]) - Mi[s]);
  });
}

// Exchange over one chunk, row normalisation: rr += w and accr[s] += w
// (m_j[s] - M_i[s]); the caller divides by r_i = rr summed over all chunks.
template <int DIM, int SMAX, int NK = 16>
__device__ __forceinline__ void exchange_chunk_row(const float (&xj)[DIM], const float (&xi)[DIM],
                                                   const float (&mj)[SMAX], const float (&Mi)[SMAX], float rc2,
                                                   float esc, bool act, float& rr, float (&accr)[SMAX]) {
  Steps<0, NK>::run([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const float w = row_weight<K, DIM>(xj, xi, rc2, esc, act);
    rr += w;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) accr[s] += w * (rshare<K>(mj[s]) - Mi[s]);
  });
}

}  // namespace rwpt
