// rwpt_layout.h -- particle-major device layouts of the positions and masses
// (internal to the HIP kernels).
//
// Positions: coordinate k of particle p at pos[d * p + k] (packed, no padding:
// a 3-D binary32 particle is one 12-byte load).  Masses: species s of
// particle p at mass[SP * p + s], SP = 2, 4 or 8 species slots (the unused
// slots hold zeros).  Gathers of a neighbour are then one or two vector loads
// instead of one load per component.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rwpt {

template <typename T, int N>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(N)));
};
template <int DIM>
constexpr int pos_stride() { return DIM; }

// Three packed coordinates (one vector load or store of 3 x sizeof(T) bytes).
template <typename T>
struct __attribute__((packed, aligned(sizeof(T)))) Packed3 {
  T x, y, z;
};

template <typename T, int DIM>
__device__ __forceinline__ void load_pos(const T* __restrict__ pos, int64_t j, T x[DIM]) {
  if constexpr (DIM == 1) {
    x[0] = pos[j];
  } else if constexpr (DIM == 2) {
    const typename VecOf<T, 2>::type v = *(const typename VecOf<T, 2>::type*)(pos + 2 * j);
    x[0] = v.x;
    x[1] = v.y;
  } else {
    const Packed3<T> v = *(const Packed3<T>*)(pos + 3 * j);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
  }
}

template <typename T, int DIM>
__device__ __forceinline__ void store_pos(T* __restrict__ pos, int64_t j, const T x[DIM]) {
  if constexpr (DIM == 1) {
    pos[j] = x[0];
  } else if constexpr (DIM == 2) {
    typename VecOf<T, 2>::type v;
    v.x = x[0];
    v.y = x[1];
    *(typename VecOf<T, 2>::type*)(pos + 2 * j) = v;
  } else {
    Packed3<T> v;
    v.x = x[0];
    v.y = x[1];
    v.z = x[2];
    *(Packed3<T>*)(pos + 3 * j) = v;
  }
}

template <typename T, int SP>
__device__ __forceinline__ void load_mass(const T* __restrict__ m, int64_t j, T out[SP]) {
  static_assert(SP == 2 || SP == 4 || SP == 8, "species slots");
  if constexpr (SP == 2) {
    const typename VecOf<T, 2>::type v = *(const typename VecOf<T, 2>::type*)(m + 2 * j);
    out[0] = v.x;
    out[1] = v.y;
  } else {
#pragma unroll
    for (int h = 0; h < SP; h += 4) {
      const typename VecOf<T, 4>::type v = *(const typename VecOf<T, 4>::type*)(m + SP * j + h);
      out[h] = v.x;
      out[h + 1] = v.y;
      out[h + 2] = v.z;
      out[h + 3] = v.w;
    }
  }
}

template <typename T, int SP>
__device__ __forceinline__ void store_mass(T* __restrict__ m, int64_t j, const T in[SP]) {
  static_assert(SP == 2 || SP == 4 || SP == 8, "species slots");
  if constexpr (SP == 2) {
    typename VecOf<T, 2>::type v;
    v.x = in[0];
    v.y = in[1];
    *(typename VecOf<T, 2>::type*)(m + 2 * j) = v;
  } else {
#pragma unroll
    for (int h = 0; h < SP; h += 4) {
      typename VecOf<T, 4>::type v;
      v.x = in[h];
      v.y = in[h + 1];
      v.z = in[h + 2];
      v.w = in[h + 3];
      *(typename VecOf<T, 4>::type*)(m + SP * j + h) = v;
    }
  }
}

// Species slots per particle for S species.
__host__ __device__ constexpr int species_slots(int S) { return S <= 2 ? 2 : (S <= 4 ? 4 : 8); }

}  // namespace rwpt
