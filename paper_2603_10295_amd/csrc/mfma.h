// The 16x16x4 matrix-core instructions of gfx950 for FP32 and FP64 operands.
#pragma once

namespace ephw {

template <typename T>
struct Mfma;
// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  They differ in where the 16x16 result lands: the f32 form gives
// lane group g = lane/16 the four consecutive rows 4g..4g+3 (register v holds
// row 4g + v), the f64 form gives it rows g, g+4, g+8, g+12 (row g + 4v).
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

}  // namespace ephw
