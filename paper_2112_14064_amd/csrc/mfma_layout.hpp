// Lane layouts of the gfx950 matrix instructions used by the front kernels,
// D(16x16) = A(16x4) B(4x16) + C: every lane supplies one element of A and of
// B and holds four elements of C/D.  Both layouts were measured on the device
// (known A, B; every candidate mapping of the accumulator compared).  Kept in
// one place so that the kernels agree.
#pragma once
#include <hip/hip_runtime.h>

namespace riga {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// A operand: lane supplies A[mfma_a_row(lane)][mfma_ab_k(lane)]
__device__ __forceinline__ int mfma_a_row(int lane) { return lane & 15; }
// B operand: lane supplies B[mfma_ab_k(lane)][mfma_b_col(lane)]
__device__ __forceinline__ int mfma_b_col(int lane) { return lane & 15; }
__device__ __forceinline__ int mfma_ab_k(int lane) { return lane >> 4; }
__device__ __forceinline__ int mfma_d_col(int lane) { return lane & 15; }

// Per element type: the 16x16x4 instruction and the accumulator row of
// element v of a lane (column is mfma_d_col for both).
template <class T> struct Mfma;

// v_mfma_f64_16x16x4_f64: lane group g = lane/16 holds rows g, g+4, g+8, g+12
template <> struct Mfma<double> {
  typedef dvec4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// v_mfma_f32_16x16x4_f32 (FP32 products, FP32 accumulation): lane group g
// holds the four consecutive rows 4g .. 4g+3
template <> struct Mfma<float> {
  typedef fvec4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

}  // namespace riga
