// Forward and backward sweeps with the multifrontal factor (Sec. 5.2.2: one
// forward/backward elimination per Arnoldi step, line 8 of Alg. 2).
//
// The factorization leaves, per node, F = [L_oo^{-1}; L_bo L_oo^{-1}]
// (nf x no, column-major) and its transpose.  With the front vector f (own
// entries of the right-hand side plus the children's update vectors):
//   forward   y_own = L_oo^{-1} f_own,   upd_v = f_bnd - (L_bo L_oo^{-1}) f_own
//             i.e. one product F f_own;
//   backward  x_own = L_oo^{-T} (y_own - L_bo^T x_bnd)
//                   = L_oo^{-T} y_own - (L_bo L_oo^{-1})^T x_bnd
//             i.e. one product F^T [y_own; -x_bnd].
// Every node is therefore a single matrix-vector product with no dependency
// chain inside it; only the tree levels are sequential.  A node's rows are split
// into tasks of 64 rows (one workgroup each: lane = row, the 8 waves take
// interleaved 8-column chunks, partial sums combined in LDS), so every load of
// F is coalesced and each row has many loads in flight; up to 4 right-hand
// sides share every load.
// The forward pass gathers children's vectors instead of scattering into
// shared boundary entries, so neither sweep needs atomics and results are
// bitwise reproducible.
#include "kernels.hpp"

namespace riga {

constexpr int ST = 512;           // threads per task: 8 waves
constexpr int SR = 64;            // rows per task: one per lane
constexpr int SC = 8;             // consecutive columns per wave and round
constexpr int SW = ST / 64;

// acc[q] of row `lane` summed over the waves through LDS; wave 0 ends with the
// total for its lane.
template <int NR>
__device__ __forceinline__ void reduce_waves(double (&acc)[NR], double* red, int lane, int wave) {
#pragma unroll
  for (int q = 0; q < NR; ++q) red[(wave * SR + lane) * NR + q] = acc[q];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double s2 = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < SW; ++w2) s2 += red[(w2 * SR + lane) * NR + q];
      acc[q] = s2;
    }
  }
}

template <int NR>
__global__ __launch_bounds__(ST) void k_fwd(DevTree t, const int4* __restrict__ tasks,
                                            const double* __restrict__ Lbuf,
                                            const double* __restrict__ b, int64_t ldb,
                                            double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ upd) {
  extern __shared__ double shm[];
  double* f = shm;                       // f[pos * NR + q], front vector
  const int4 tk = tasks[blockIdx.x];
  const int v = tk.x, r0 = tk.y, r1 = tk.z;
  const int nf = t.nf[v], no = t.no[v];
  double* red = shm + (size_t)nf * NR;   // SW x SR x NR partial sums
  const double* F = Lbuf + t.loff[v];
  const int* fd = t.fdofs + t.foff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int p = tid; p < nf; p += ST)
#pragma unroll
    for (int q = 0; q < NR; ++q) f[p * NR + q] = (p < no) ? b[fd[p] + q * ldb] : 0.0;
  __syncthreads();
  for (int ci = t.coff[v]; ci < t.coff[v + 1]; ++ci) {
    const int c = t.clist[ci];
    const int nbc = t.nb[c];
    const int* mp = t.maps + t.moff[c];
    const double* uc = upd + (int64_t)t.voff[c] * NR;
    for (int k = tid; k < nbc; k += ST)
#pragma unroll
      for (int q = 0; q < NR; ++q) f[mp[k] * NR + q] += uc[k * NR + q];
    __syncthreads();
  }
  const int r = r0 + lane;
  const bool live = r < r1;
  // columns past the diagonal of L_oo^{-1} are exact zeros: an own-row block
  // stops at its last row's diagonal
  const int jend = (r1 - 1 < no) ? r1 : no;
  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  const double* col = F + (live ? r : r0);
  for (int j0 = wave * SC; j0 < jend; j0 += SW * SC) {
    double a[SC];
#pragma unroll
    for (int u = 0; u < SC; ++u) a[u] = (j0 + u < jend) ? col[(int64_t)(j0 + u) * nf] : 0.0;
#pragma unroll
    for (int u = 0; u < SC; ++u) {
      const int j = min(j0 + u, jend - 1);
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] += a[u] * f[j * NR + q];
    }
  }
  reduce_waves<NR>(acc, red, lane, wave);
  if (wave == 0 && live) {
    if (r < no) {
#pragma unroll
      for (int q = 0; q < NR; ++q) y[fd[r] + q * ldy] = acc[q];
    } else {
      double* uv = upd + (int64_t)(t.voff[v] + r - no) * NR;
#pragma unroll
      for (int q = 0; q < NR; ++q) uv[q] = f[r * NR + q] - acc[q];
    }
  }
}

template <int NR>
__global__ __launch_bounds__(ST) void k_bwd(DevTree t, const int4* __restrict__ tasks,
                                            const double* __restrict__ Tbuf,
                                            const double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ x, int64_t ldx,
                                            double* __restrict__ r_l, const double* __restrict__ v_u,
                                            int64_t ldv, double sig) {
  extern __shared__ double shm[];
  double* w = shm;                       // [y_own; -x_bnd]
  const int4 tk = tasks[blockIdx.x];
  const int v = tk.x, a0 = tk.y, a1 = tk.z;
  const int nf = t.nf[v], no = t.no[v];
  double* red = shm + (size_t)nf * NR;
  const double* T = Tbuf + t.loff[v];   // element (a, i) of F^T at T[i * no + a]
  const int* fd = t.fdofs + t.foff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool epilogue = (r_l != nullptr);

  for (int p = tid; p < nf; p += ST)
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double val;
      if (p < no) {
        val = y[fd[p] + q * ldy];
      } else {
        val = x[fd[p] + q * ldx];
        if (!epilogue) val = -val;   // with the epilogue, ancestors stored r_u = -x already
      }
      w[p * NR + q] = val;
    }
  __syncthreads();
  const int a = a0 + lane;
  const bool live = a < a1;
  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  // entries above the diagonal of L_oo^{-T} vanish: start at the block's first row
  const double* row = T + (live ? a : a0);
  for (int i0 = a0 + wave * SC; i0 < nf; i0 += SW * SC) {
    double e[SC];
#pragma unroll
    for (int u = 0; u < SC; ++u) e[u] = (i0 + u < nf) ? row[(int64_t)(i0 + u) * no] : 0.0;
#pragma unroll
    for (int u = 0; u < SC; ++u) {
      const int i = min(i0 + u, nf - 1);
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] += e[u] * w[i * NR + q];
    }
  }
  reduce_waves<NR>(acc, red, lane, wave);
  if (wave == 0 && live) {
    const int d = fd[a];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if (epilogue) {
        const double ru = -acc[q];
        x[d + q * ldx] = ru;
        r_l[d + q * ldx] = sig * ru + v_u[d + q * ldv];
      } else {
        x[d + q * ldx] = acc[q];
      }
    }
  }
}

void launch_fwd_level(const DevTree& t, const int4* tasks, int count, int nrhs, const double* L,
                      const double* b, int64_t ldb, double* y, int64_t ldy, double* upd, int max_front,
                      hipStream_t st) {
  if (count <= 0) return;
  size_t shm = ((size_t)max_front + SW * SR) * nrhs * sizeof(double);
#define RIGA_FWD(NR) \
  hipLaunchKernelGGL(k_fwd<NR>, dim3(count), dim3(ST), shm, st, t, tasks, L, b, ldb, y, ldy, upd)
  switch (nrhs) {
    case 1: RIGA_FWD(1); break;
    case 2: RIGA_FWD(2); break;
    case 3: RIGA_FWD(3); break;
    default: RIGA_FWD(4); break;
  }
#undef RIGA_FWD
}

void launch_bwd_level(const DevTree& t, const int4* tasks, int count, int nrhs, const double* T,
                      const double* y, int64_t ldy, double* x, int64_t ldx, double* r_l, const double* v_u,
                      int64_t ldv, double sig, int max_front, hipStream_t st) {
  if (count <= 0) return;
  size_t shm = ((size_t)max_front + SW * SR) * nrhs * sizeof(double);
#define RIGA_BWD(NR)                                                                               \
  hipLaunchKernelGGL(k_bwd<NR>, dim3(count), dim3(ST), shm, st, t, tasks, T, y, ldy, x, ldx, r_l, v_u, \
                     ldv, sig)
  switch (nrhs) {
    case 1: RIGA_BWD(1); break;
    case 2: RIGA_BWD(2); break;
    case 3: RIGA_BWD(3); break;
    default: RIGA_BWD(4); break;
  }
#undef RIGA_BWD
}

}  // namespace riga
