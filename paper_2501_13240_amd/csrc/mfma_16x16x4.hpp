// 16x16x4 matrix-core products in FP64 and FP32 (internal), shared by the
// tensor-product kernels that contract small dense matrices with element
// blocks.  Operand layout of one product C += A B (A 16x4, B 4x16): lane
// i + 16 k holds A[i][k] and B[k][i]; result (i, j) sits in lane
// 16 (i % 4) + j, register i / 4 (FP64) or lane 16 (i / 4) + j, register
// i % 4 (FP32).
#pragma once

#include <hip/hip_runtime.h>

namespace sem {

typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mm;
template <>
struct Mm<double> {
  typedef v4d_t V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the result held in register r of this lane
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mm<float> {
  typedef v4f_t V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

}  // namespace sem
