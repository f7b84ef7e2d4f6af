// Lane layout of the gfx950 FP64 matrix instruction v_mfma_f64_16x16x4_f64,
// D(16x16) = A(16x4) B(4x16) + C: every lane supplies one element of A and of
// B and holds four elements of C/D.  Kept in one place so that the kernels and
// the layout self-test agree.
#pragma once
#include <hip/hip_runtime.h>

namespace riga {

typedef double dvec4 __attribute__((ext_vector_type(4)));

// A operand: lane supplies A[mfma_a_row(lane)][mfma_ab_k(lane)]
__device__ __forceinline__ int mfma_a_row(int lane) { return lane & 15; }
// B operand: lane supplies B[mfma_ab_k(lane)][mfma_b_col(lane)]
__device__ __forceinline__ int mfma_b_col(int lane) { return lane & 15; }
__device__ __forceinline__ int mfma_ab_k(int lane) { return lane >> 4; }
// accumulator: element v of the lane's dvec4 is D[mfma_d_row(lane, v)][mfma_d_col(lane)]
// (rows interleave: lane group g = lane/16 holds rows g, g+4, g+8, g+12)
__device__ __forceinline__ int mfma_d_row(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int mfma_d_col(int lane) { return lane & 15; }

}  // namespace riga
