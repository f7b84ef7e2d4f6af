// Device bodies shared by the single-problem and the batched Krylov kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace riga {

// End of a block Gram--Schmidt step for one problem (see k_block_normalize):
// H[0:nc, k+q] = h1 + h2, G = R^T R, H[nc+c, k+q] = R[c][q], Rinv = R^{-1};
// *flag = 1 when a column lost its norm.  Called by every thread of a block;
// hn: 4 doubles of shared memory.
__device__ inline void block_normalize_body(int nc, int nq, const double* h1, const double* h2, const double* G,
                                            double* H, int ldh, int k, double* Rinv, int* flag, double* hn) {
  for (int idx = threadIdx.x; H && idx < nc * nq; idx += blockDim.x) {
    const int c = idx / nq, q = idx % nq;
    H[c + (int64_t)(k + q) * ldh] = (h1 ? h1[idx] : 0.0) + (h2 ? h2[idx] : 0.0);
  }
  // squared norms of the projection coefficients, one wave per column q
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv < nq) {
    double sacc = 0.0;
    for (int c = lane; c < nc; c += 64) {
      const double hv = (h1 ? h1[c * nq + wv] : 0.0) + (h2 ? h2[c * nq + wv] : 0.0);
      sacc += hv * hv;
    }
    for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
    if (lane == 0) hn[wv] = sacc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double R[4][4] = {{0}}, X[4][4] = {{0}};
  bool bad = false;
  for (int j = 0; j < nq; ++j) {
    const double n0 = G[j * nq + j] + hn[j];
    for (int i = 0; i <= j; ++i) {
      double sacc = 0.5 * (G[i * nq + j] + G[j * nq + i]);
      for (int kk = 0; kk < i; ++kk) sacc -= R[kk][i] * R[kk][j];
      if (i == j) {
        if (!(sacc > 1e-24 * n0)) { bad = true; sacc = 1.0; }
        R[j][j] = sqrt(sacc);
      } else {
        R[i][j] = sacc / R[i][i];
      }
    }
  }
  for (int j = 0; j < nq; ++j) {
    X[j][j] = 1.0 / R[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double sacc = 0.0;
      for (int kk = i + 1; kk <= j; ++kk) sacc += R[i][kk] * X[kk][j];
      X[i][j] = -sacc / R[i][i];
    }
  }
  for (int q = 0; q < nq; ++q)
    for (int c = 0; c < nq; ++c) {
      if (H) H[nc + c + (int64_t)(k + q) * ldh] = R[c][q];
      Rinv[c + q * nq] = X[c][q];
    }
  if (bad) *flag = 1;
}

constexpr int GEMM_THREADS = 256;
constexpr int GEMM_ROWS = 64;     // rows of In per tile

// Rows [r0, r0 + rows) of Out = In * Q (In n x kin with leading dimension ldi,
// Q kin x kout column-major).  The tile of In is staged in LDS (laid out
// [t][row] so the lanes of a wave read consecutive words), and so are 16
// columns of Q at a time (read as broadcasts); lane = row, every wave takes four
// of those columns.  shm: kin * 64 + kin * 16 doubles.  Called by every thread
// of a 256-thread block.
__device__ inline void gemm_tile64(int64_t r0, int rows, const double* __restrict__ In, int64_t ldi, int kin,
                                   const double* __restrict__ Q, int kout, double* __restrict__ Out,
                                   int64_t out_rs, int64_t out_cs, double* shm) {
  double* tile = shm;                         // [t][row]
  double* qs = shm + (size_t)kin * GEMM_ROWS;  // [c][t], 16 columns
  __syncthreads();   // the previous tile has been consumed
  for (int idx = threadIdx.x; idx < GEMM_ROWS * kin; idx += GEMM_THREADS) {
    const int r = idx % GEMM_ROWS, t = idx / GEMM_ROWS;
    tile[idx] = (r < rows) ? In[r0 + r + (int64_t)t * ldi] : 0.0;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int p0 = 0; p0 < kout; p0 += 16) {
    const int np = min(16, kout - p0);
    if (p0 > 0) __syncthreads();   // the previous columns of Q have been consumed
    for (int idx = threadIdx.x; idx < 16 * kin; idx += GEMM_THREADS) {
      const int c = idx / kin, t = idx % kin;
      qs[idx] = (c < np) ? Q[(int64_t)(p0 + c) * kin + t] : 0.0;
    }
    __syncthreads();
    const int c0 = wave * 4;
    if (c0 >= np) continue;
    const double* q = qs + (size_t)c0 * kin;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < kin; ++t) {
      const double a = tile[t * GEMM_ROWS + lane];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += a * q[u * kin + t];
    }
    if (lane < rows)
      for (int u = 0; u < min(4, np - c0); ++u) Out[(r0 + lane) * out_rs + (int64_t)(p0 + c0 + u) * out_cs] = acc[u];
  }
}

}  // namespace riga
