// The 16x16x4 matrix-core product of gfx950 in FP64 and FP32: D += A B with
// A 16 x 4 (lane l holds A[l % 16][l / 16]), B 4 x 16 (lane l holds
// B[l / 16][l % 16]) and D 16 x 16, four values per lane in column l % 16 at
// the rows given by row(l, v) (the two precisions order them differently).
#pragma once

#include <hip/hip_runtime.h>

namespace qgw {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of D held in element v by lane l (column l % 16)
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

}  // namespace qgw
