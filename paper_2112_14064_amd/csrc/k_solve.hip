// Forward and backward sweeps with the multifrontal factor (Sec. 5.2.2: one
// forward/backward elimination per Arnoldi step, line 8 of Alg. 2).
//
// Forward (leaves to root), per node v, front vector f (own then boundary):
//   f_own = b[own] + sum of the children's update vectors mapped into the front,
//   y_own = L_oo^{-1} f_own,   upd_v = f_bnd - L_bo y_own  (kept for the parent).
// Backward (root to leaves):
//   x_own = L_oo^{-T} (y_own - L_bo^T x[bnd]).
// The forward pass gathers children's vectors instead of scattering into shared
// boundary entries, so neither sweep needs atomics and results are bitwise
// reproducible.  One workgroup per node; up to 4 right-hand sides share every
// read of the factor.
#include "kernels.hpp"

namespace riga {

constexpr int ST = 256;
constexpr int SW = 16;   // substitution panel width

template <int NR>
__global__ __launch_bounds__(ST) void k_fwd(DevTree t, const int* __restrict__ level_nodes,
                                            const double* __restrict__ Lbuf,
                                            const double* __restrict__ b, int64_t ldb,
                                            double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ upd) {
  extern __shared__ double f[];   // f[pos * NR + q]
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v], nb = t.nb[v];
  const double* L = Lbuf + t.loff[v];
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

  for (int k0 = 0; k0 < no; k0 += SW) {
    const int w = min(SW, no - k0);
    // diagonal block: lane (q, r) holds row r of the block for right-hand side q
    if (wave == 0 && lane < SW * NR) {
      const int r = lane % SW, q = lane / SW;
      double row[SW];
#pragma unroll
      for (int c = 0; c < SW; ++c) row[c] = (r < w && c <= r) ? L[(int64_t)(k0 + c) * nf + k0 + r] : 0.0;
      double fr = (r < w) ? f[(k0 + r) * NR + q] : 0.0;
#pragma unroll
      for (int c = 0; c < SW; ++c) {
        if (c < w) {
          if (r == c) fr = fr / row[c];
          double yc = __shfl(fr, q * SW + c, 64);
          if (r > c) fr -= row[c] * yc;
        }
      }
      if (r < w) f[(k0 + r) * NR + q] = fr;
    }
    __syncthreads();
    // rows below the block
    for (int i = k0 + w + tid; i < nf; i += ST) {
      double acc[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] = f[i * NR + q];
#pragma unroll
      for (int c = 0; c < SW; ++c) {
        if (c < w) {
          double l = L[(int64_t)(k0 + c) * nf + i];
#pragma unroll
          for (int q = 0; q < NR; ++q) acc[q] -= l * f[(k0 + c) * NR + q];
        }
      }
#pragma unroll
      for (int q = 0; q < NR; ++q) f[i * NR + q] = acc[q];
    }
    __syncthreads();
  }
  for (int p = tid; p < no; p += ST)
#pragma unroll
    for (int q = 0; q < NR; ++q) y[fd[p] + q * ldy] = f[p * NR + q];
  double* uv = upd + (int64_t)t.voff[v] * NR;
  for (int k = tid; k < nb; k += ST)
#pragma unroll
    for (int q = 0; q < NR; ++q) uv[k * NR + q] = f[(no + k) * NR + q];
}

template <int NR>
__device__ __forceinline__ void wave_sum(double (&a)[NR]) {
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a[q] += __shfl_xor(a[q], off, 64);
}

template <int NR>
__global__ __launch_bounds__(ST) void k_bwd(DevTree t, const int* __restrict__ level_nodes,
                                            const double* __restrict__ Lbuf,
                                            const double* __restrict__ y, int64_t ldy,
                                            double* __restrict__ x, int64_t ldx,
                                            double* __restrict__ r_l, const double* __restrict__ v_u,
                                            int64_t ldv, double sig) {
  extern __shared__ double s[];   // s[pos * NR + q]: own rhs / solution, then x on the boundary
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v], nb = t.nb[v];
  const double* L = Lbuf + t.loff[v];
  const int* fd = t.fdofs + t.foff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool epilogue = (r_l != nullptr);

  for (int p = tid; p < nf; p += ST)
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double val;
      if (p < no) val = y[fd[p] + q * ldy];
      else {
        val = x[fd[p] + q * ldx];
        if (epilogue) val = -val;   // ancestors stored r_u = -x
      }
      s[p * NR + q] = val;
    }
  __syncthreads();
  // own -= L_bo^T x_bnd: one wave per column, lanes along the column
  if (nb > 0) {
    for (int a = wave; a < no; a += ST / 64) {
      double acc[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[q] = 0.0;
      const double* col = L + (int64_t)a * nf + no;
      for (int k = lane; k < nb; k += 64) {
        double l = col[k];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] += l * s[(no + k) * NR + q];
      }
      wave_sum<NR>(acc);
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < NR; ++q) s[a * NR + q] -= acc[q];
    }
    __syncthreads();
  }
  const int last = ((no - 1) / SW) * SW;
  for (int k0 = last; k0 >= 0 && no > 0; k0 -= SW) {
    const int w = min(SW, no - k0);
    // subtract the already solved own rows below the block
    if (k0 + w < no) {
      for (int a = k0 + wave; a < k0 + w; a += ST / 64) {
        double acc[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = 0.0;
        const double* col = L + (int64_t)a * nf;
        for (int i = k0 + w + lane; i < no; i += 64) {
          double l = col[i];
#pragma unroll
          for (int q = 0; q < NR; ++q) acc[q] += l * s[i * NR + q];
        }
        wave_sum<NR>(acc);
        if (lane == 0)
#pragma unroll
          for (int q = 0; q < NR; ++q) s[a * NR + q] -= acc[q];
      }
      __syncthreads();
    }
    // transposed diagonal block: lane (q, r) holds column r of the block
    if (wave == 0 && lane < SW * NR) {
      const int r = lane % SW, q = lane / SW;
      double col[SW];
#pragma unroll
      for (int c = 0; c < SW; ++c) col[c] = (r < w && c >= r && c < w) ? L[(int64_t)(k0 + r) * nf + k0 + c] : 0.0;
      double tr = (r < w) ? s[(k0 + r) * NR + q] : 0.0;
#pragma unroll
      for (int c = SW - 1; c >= 0; --c) {
        if (c < w) {
          if (r == c) tr = tr / col[c];
          double xc = __shfl(tr, q * SW + c, 64);
          if (r < c) tr -= col[c] * xc;
        }
      }
      if (r < w) s[(k0 + r) * NR + q] = tr;
    }
    __syncthreads();
  }
  for (int p = tid; p < no; p += ST) {
    const int d = fd[p];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double val = s[p * NR + q];
      if (epilogue) {
        double ru = -val;
        x[d + q * ldx] = ru;
        r_l[d + q * ldx] = sig * ru + v_u[d + q * ldv];
      } else {
        x[d + q * ldx] = val;
      }
    }
  }
}

void launch_fwd_level(const DevTree& t, const int* level_nodes, int count, int nrhs,
                      const double* L, const double* b, int64_t ldb, double* y, int64_t ldy,
                      double* upd, int max_front, hipStream_t st) {
  if (count <= 0) return;
  size_t shm = (size_t)max_front * nrhs * sizeof(double);
  switch (nrhs) {
    case 1: hipLaunchKernelGGL(k_fwd<1>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, b, ldb, y, ldy, upd); break;
    case 2: hipLaunchKernelGGL(k_fwd<2>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, b, ldb, y, ldy, upd); break;
    case 3: hipLaunchKernelGGL(k_fwd<3>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, b, ldb, y, ldy, upd); break;
    default: hipLaunchKernelGGL(k_fwd<4>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, b, ldb, y, ldy, upd); break;
  }
}

void launch_bwd_level(const DevTree& t, const int* level_nodes, int count, int nrhs,
                      const double* L, const double* y, int64_t ldy, double* x, int64_t ldx,
                      double* r_l, const double* v_u, int64_t ldv, double sig,
                      int max_front, hipStream_t st) {
  if (count <= 0) return;
  size_t shm = (size_t)max_front * nrhs * sizeof(double);
  switch (nrhs) {
    case 1: hipLaunchKernelGGL(k_bwd<1>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, y, ldy, x, ldx, r_l, v_u, ldv, sig); break;
    case 2: hipLaunchKernelGGL(k_bwd<2>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, y, ldy, x, ldx, r_l, v_u, ldv, sig); break;
    case 3: hipLaunchKernelGGL(k_bwd<3>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, y, ldy, x, ldx, r_l, v_u, ldv, sig); break;
    default: hipLaunchKernelGGL(k_bwd<4>, dim3(count), dim3(ST), shm, st, t, level_nodes, L, y, ldy, x, ldx, r_l, v_u, ldv, sig); break;
  }
}

}  // namespace riga
