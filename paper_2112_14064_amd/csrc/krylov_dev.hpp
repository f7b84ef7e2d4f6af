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
constexpr int GEMM_CHUNK = 32;
constexpr int GEMM_UNROLL = 8;

// Row i of Out = In * Q (In n x kin with leading dimension ldi, Q kin x kout
// column-major) for the rows of one workgroup; every thread of the block
// calls it (live = false for threads past the rows).  qs: kin * 32 doubles of
// shared memory.  32 output columns per pass kept in registers; the inner loop
// issues 8 independent coalesced loads of In before using them.
__device__ inline void gemm_tall_row(int64_t i, bool live, const double* __restrict__ In, int64_t ldi, int kin,
                                     const double* __restrict__ Q, int kout, double* __restrict__ Out,
                                     int64_t out_rs, int64_t out_cs, double* qs) {
  for (int c0 = 0; c0 < kout; c0 += GEMM_CHUNK) {
    const int kc = min(GEMM_CHUNK, kout - c0);
    __syncthreads();
    for (int k = threadIdx.x; k < kin * GEMM_CHUNK; k += GEMM_THREADS) {
      const int tt = k / GEMM_CHUNK, c = k % GEMM_CHUNK;
      qs[k] = (c < kc) ? Q[(int64_t)(c0 + c) * kin + tt] : 0.0;
    }
    __syncthreads();
    if (!live) continue;
    double acc[GEMM_CHUNK];
#pragma unroll
    for (int c = 0; c < GEMM_CHUNK; ++c) acc[c] = 0.0;
    for (int t0 = 0; t0 < kin; t0 += GEMM_UNROLL) {
      double a[GEMM_UNROLL];
#pragma unroll
      for (int u = 0; u < GEMM_UNROLL; ++u) a[u] = (t0 + u < kin) ? In[i + (int64_t)(t0 + u) * ldi] : 0.0;
#pragma unroll
      for (int u = 0; u < GEMM_UNROLL; ++u) {
        const int tt = min(t0 + u, kin - 1);
#pragma unroll
        for (int c = 0; c < GEMM_CHUNK; ++c) acc[c] += a[u] * qs[tt * GEMM_CHUNK + c];
      }
    }
#pragma unroll
    for (int c = 0; c < GEMM_CHUNK; ++c)
      if (c < kc) Out[i * out_rs + (int64_t)(c0 + c) * out_cs] = acc[c];
  }
}

}  // namespace riga
