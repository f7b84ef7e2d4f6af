// Multifrontal Cholesky of Q(sigma) = sigma^2 M + sigma C + K over the
// nested-dissection tree (Sec. 3.3: rIGA hyperplanes are the separators;
// Sec. 5.2.1: one factorization per shift).
//
// A front of node v holds its own dofs (eliminated here) followed by its
// boundary dofs (ancestors coupled to the subtree).  Storage per node:
//   L block  nf x no, column-major (ld nf): columns of the factor for the own
//            dofs, rows own+boundary.
//   U block  nb x nb, column-major: the update (Schur complement) matrix that
//            the parent adds into its front ("extend-add").
// One workgroup per front.  The own block is factored by a right-looking
// blocked Cholesky with 16-wide panels: the diagonal 16x16 block by one wave in
// LDS, the panel below by a row-parallel triangular solve, and the trailing
// lower triangle (including the update block) by FP64 MFMA 16x16x4 tiles.
#include "kernels.hpp"
#include "mfma_layout.hpp"

namespace riga {

constexpr int FT = 256;   // threads per front
constexpr int PW = 16;    // panel width = MFMA tile

struct Front {
  double* L; double* U; int nf, no, nb;
  __device__ __forceinline__ double* at(int i, int j) const {  // requires i >= j
    return j < no ? L + (int64_t)j * nf + i : U + (int64_t)(j - no) * nb + (i - no);
  }
};

__global__ __launch_bounds__(FT) void k_front_factor(
    int n, const int* __restrict__ lo, const int* __restrict__ hi, const int64_t* __restrict__ rowptr,
    DevTree t, const int* __restrict__ level_nodes, double s2, double s1,
    const double* __restrict__ Kv, const double* __restrict__ Mv, const double* __restrict__ Cv,
    double* __restrict__ Lbuf, double* __restrict__ Ubuf, int64_t* __restrict__ status) {
  const int v = level_nodes[blockIdx.x];
  Front F{Lbuf + t.loff[v], Ubuf + t.uoff[v], t.nf[v], t.no[v], t.nb[v]};
  const int nf = F.nf, no = F.no, nb = F.nb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int* fd = t.fdofs + t.foff[v];
  const int* fk = t.fkey + t.foff[v];
  const int* fp = t.fpos + t.foff[v];

  // --- A: clear the front -------------------------------------------------------
  for (int64_t idx = tid; idx < (int64_t)nf * no; idx += FT) F.L[idx] = 0.0;
  for (int64_t idx = tid; idx < (int64_t)nb * nb; idx += FT) F.U[idx] = 0.0;
  __syncthreads();

  // --- B: original entries Q[g, d] for own d, g in the front, g at or below d ----
  for (int a = tid; a < no; a += FT) {
    const int d = fd[a];
    const int i = d % n, j = d / n;
    const int wx = hi[i] - lo[i] + 1;
    const int64_t k0 = rowptr[d], k1 = rowptr[d + 1];
    for (int64_t k = k0; k < k1; ++k) {
      const int o = (int)(k - k0);
      const int g = (lo[j] + o / wx) * n + lo[i] + o % wx;
      int x0 = 0, x1 = nf;  // binary search g in the sorted front keys
      while (x1 - x0 > 1) {
        int c = (x0 + x1) >> 1;
        if (fk[c] <= g) x0 = c; else x1 = c;
      }
      if (nf > 0 && fk[x0] == g) {
        const int pos = fp[x0];
        if (pos >= a) *F.at(pos, a) = s2 * Mv[k] + s1 * Cv[k] + Kv[k];
      }
    }
  }
  __syncthreads();

  // --- C: extend-add of the children's update blocks ------------------------------
  for (int ci = t.coff[v]; ci < t.coff[v + 1]; ++ci) {
    const int c = t.clist[ci];
    const int nbc = t.nb[c];
    const double* Uc = Ubuf + t.uoff[c];
    const int* mp = t.maps + t.moff[c];
    for (int64_t idx = tid; idx < (int64_t)nbc * nbc; idx += FT) {
      const int l = (int)(idx / nbc), k = (int)(idx % nbc);
      if (k >= l) *F.at(mp[k], mp[l]) += Uc[idx];
    }
    __syncthreads();
  }

  // --- D: partial Cholesky of the own columns --------------------------------------
  __shared__ double dg[PW][PW + 1];
  for (int k0 = 0; k0 < no; k0 += PW) {
    const int w = min(PW, no - k0);
    // D1: diagonal block by wave 0 (wave-synchronous LDS)
    if (wave == 0) {
      for (int idx = lane; idx < PW * PW; idx += 64) {
        int r = idx / PW, c = idx % PW;
        dg[r][c] = (r < w && c <= r) ? *F.at(k0 + r, k0 + c) : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int c = 0; c < w; ++c) {
        double piv = dg[c][c];
        if (!(piv > 0.0)) {           // not SPD (or NaN): record, continue with 1
          if (lane == 0) atomicCAS((unsigned long long*)status, (unsigned long long)(-1ll),
                                   (unsigned long long)fd[k0 + c]);
          piv = 1.0;
        }
        const double dd = sqrt(piv), inv = 1.0 / dd;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane > c && lane < w) dg[lane][c] *= inv;
        if (lane == c) dg[c][c] = dd;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // rank-1 update of the remaining lower triangle (r, cc), c < cc <= r < w
        for (int idx = lane; idx < PW * PW; idx += 64) {
          int r = idx / PW, cc = idx % PW;
          if (r < w && cc > c && cc <= r) dg[r][cc] -= dg[r][c] * dg[cc][c];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      for (int idx = lane; idx < PW * PW; idx += 64) {
        int r = idx / PW, c = idx % PW;
        if (r < w && c <= r) *F.at(k0 + r, k0 + c) = dg[r][c];
      }
    }
    __syncthreads();
    // D2: panel rows below the diagonal block: x L_kk^T = a
    for (int i = k0 + w + tid; i < nf; i += FT) {
      double x[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) x[c] = (c < w) ? F.L[(int64_t)(k0 + c) * nf + i] : 0.0;
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        if (c < w) {
          double s = x[c];
#pragma unroll
          for (int c2 = 0; c2 < PW; ++c2)
            if (c2 < c) s -= x[c2] * dg[c][c2];
          x[c] = s / dg[c][c];
        }
      }
#pragma unroll
      for (int c = 0; c < PW; ++c)
        if (c < w) F.L[(int64_t)(k0 + c) * nf + i] = x[c];
    }
    __syncthreads();
    // D3: trailing update A22 -= P P^T on the lower triangle, 16x16 MFMA tiles
    const int s0 = k0 + w;
    const int nt = (nf - s0 + PW - 1) / PW;
    const int ntiles = nt * (nt + 1) / 2;
    for (int tile = wave; tile < ntiles; tile += FT / 64) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= tile) ++I;
      const int J = tile - I * (I + 1) / 2;
      const int rI = s0 + PW * I, rJ = s0 + PW * J;
      dvec4 acc;
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        int r = rI + mfma_d_row(lane, vv), c = rJ + mfma_d_col(lane);
        acc[vv] = (r < nf && c < nf && r >= c) ? *F.at(r, c) : 0.0;
      }
#pragma unroll
      for (int kk = 0; kk < PW / 4; ++kk) {
        const int pc = 4 * kk + mfma_ab_k(lane);     // panel column
        const int ra = rI + mfma_a_row(lane), rb = rJ + mfma_b_col(lane);
        double av = 0.0, bv = 0.0;
        if (pc < w) {
          if (ra < nf) av = -F.L[(int64_t)(k0 + pc) * nf + ra];
          if (rb < nf) bv = F.L[(int64_t)(k0 + pc) * nf + rb];
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        int r = rI + mfma_d_row(lane, vv), c = rJ + mfma_d_col(lane);
        if (r < nf && c < nf && r >= c) *F.at(r, c) = acc[vv];
      }
    }
    __syncthreads();
  }
}

void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count,
                         double s2, double s1, const double* K, const double* M, const double* C,
                         double* L, double* U, int64_t* status, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_front_factor, dim3(count), dim3(FT), 0, st, s.n, s.lo, s.hi, s.rowptr, t,
                     level_nodes, s2, s1, K, M, C, L, U, status);
}

}  // namespace riga
