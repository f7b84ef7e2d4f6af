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
//
// For the solves the factor columns are then replaced by
//   F = [L_oo^{-1}; L_bo L_oo^{-1}],
// obtained row by row from X L_oo = [I; L_bo] (a triangular solve from the
// right, MFMA for the panel updates).  F is kept column-major in the L block
// and transposed (no x nf, column-major) in the T block, so each sweep of a
// forward/backward solve is one matrix-vector product per node:
//   forward   [y_own; w] = F f_own,  update to the parent = f_bnd - w
//   backward  x_own = F^T [y_own; -x_bnd].
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
    double* __restrict__ Lbuf, double* __restrict__ Ubuf, double* __restrict__ Tbuf,
    int64_t* __restrict__ status) {
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

  // --- E: X L_oo = [I; L_bo], row tiles per wave, panels from the right --------------
  double* T = Tbuf + t.loff[v];      // X row r at T[r * no + 0 .. no)
  __shared__ double tb[FT / 64][PW][PW + 1];
  __shared__ double lp[FT / 64][PW][PW + 1];
  const int npan = (no + PW - 1) / PW;
  const int nrt = (nf + PW - 1) / PW;
  for (int rt = wave; rt < nrt; rt += FT / 64) {
    const int r0 = rt * PW;
    for (int P = npan - 1; P >= 0; --P) {
      const int c0 = P * PW, w = min(PW, no - c0);
      const bool top = (r0 + PW <= no);          // every row of the tile is an own row
      if (top && r0 + PW - 1 < c0) {             // X[r][c] = 0 for c > r < no
        for (int idx = lane; idx < PW * PW; idx += 64) {
          int i = idx / PW, j = idx % PW;
          if (j < w) T[(int64_t)(r0 + i) * no + c0 + j] = 0.0;
        }
        continue;
      }
      dvec4 acc;
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int r = r0 + mfma_d_row(lane, vv), c = c0 + mfma_d_col(lane);
        double val = 0.0;
        if (r < nf && c < c0 + w) val = (r < no) ? (r == c ? 1.0 : 0.0) : F.L[(int64_t)c * nf + r];
        acc[vv] = val;
      }
      // minus X[r][k] L_oo[k][c] over the already solved columns k >= c0 + w
      const int kend = top ? min(no, r0 + PW) : no;
      for (int k0 = c0 + w; k0 < kend; k0 += 4) {
        const int ra = r0 + mfma_a_row(lane), ka = k0 + mfma_ab_k(lane);
        const int cb = c0 + mfma_b_col(lane);
        const double av = (ra < nf && ka < no) ? -T[(int64_t)ra * no + ka] : 0.0;
        const double bv = (ka < no && cb < c0 + w) ? F.L[(int64_t)cb * nf + ka] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) tb[wave][mfma_d_row(lane, vv)][mfma_d_col(lane)] = acc[vv];
      for (int idx = lane; idx < PW * PW; idx += 64) {
        int i = idx / PW, j = idx % PW;
        lp[wave][i][j] = (i < w && j <= i) ? F.L[(int64_t)(c0 + j) * nf + c0 + i] : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (lane < PW) {  // row lane: x L_PP = acc, from the last column back
        for (int j = w - 1; j >= 0; --j) {
          double sacc = tb[wave][lane][j];
          for (int k = j + 1; k < w; ++k) sacc -= tb[wave][lane][k] * lp[wave][k][j];
          tb[wave][lane][j] = sacc / lp[wave][j][j];
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int idx = lane; idx < PW * PW; idx += 64) {
        int i = idx / PW, j = idx % PW;
        if (r0 + i < nf && j < w) T[(int64_t)(r0 + i) * no + c0 + j] = tb[wave][i][j];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  // F column-major into the L block
  for (int64_t idx = tid; idx < (int64_t)nf * no; idx += FT) {
    const int r = (int)(idx % nf), a = (int)(idx / nf);
    F.L[idx] = T[(int64_t)r * no + a];
  }
}

void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count,
                         double s2, double s1, const double* K, const double* M, const double* C,
                         double* L, double* U, double* T, int64_t* status, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_front_factor, dim3(count), dim3(FT), 0, st, s.n, s.lo, s.hi, s.rowptr, t,
                     level_nodes, s2, s1, K, M, C, L, U, T, status);
}

}  // namespace riga
