// Device bodies shared by the single-problem and the batched Krylov kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"
#include "mfma_layout.hpp"

namespace riga {

// Sparse rows with the implicit tensor sparsity are summed by groups of
// SPMV_G lanes; a row of up to SPMV_U * SPMV_G stored entries (every degree
// up to 4) issues all of its loads before the first product, so a row costs
// one memory latency instead of one per round of lanes.
constexpr int SPMV_G = 16;
constexpr int SPMV_U = 6;

// s[q] += sum_o a[o] x[(o / wx) * n + o % wx + q * ldx] over this lane's
// entries o = g, g + SPMV_G, ... < len (increasing o: the order of a plain loop).
template <int NC>
__device__ __forceinline__ void tensor_row_sum(const double* __restrict__ a, int len,
                                               const double* __restrict__ x, int64_t ldx, int n, int wx, int g,
                                               double (&s)[NC]) {
  for (int o0 = 0; o0 < len; o0 += SPMV_U * SPMV_G) {
    double av[SPMV_U], xv[SPMV_U][NC];
#pragma unroll
    for (int u = 0; u < SPMV_U; ++u) {
      const int o = o0 + u * SPMV_G + g;
      if (o < len) {
        const int dy = o / wx;
        const double* xp = x + (int64_t)dy * n + (o - dy * wx);
        av[u] = a[o];
#pragma unroll
        for (int q = 0; q < NC; ++q) xv[u][q] = xp[q * ldx];
      } else {
        av[u] = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) xv[u][q] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < SPMV_U; ++u)
#pragma unroll
      for (int q = 0; q < NC; ++q) s[q] += av[u] * xv[u][q];
  }
}

// Sums over the 64 lanes of a wave of V values per lane (V a power of two,
// at most 64) by recursive halving: at exchange s (offset 32 >> s) a lane
// keeps the lower or the upper half of its values, by bit 5 - s of its lane
// index, and adds its partner's copy of that half, so log2 V exchanges move
// V - 1 values in all, and 6 - log2 V plain exchanges finish the one left.
// Lane l then holds the total of value l >> (6 - log2 V) (every lane of that
// group of 64 / V lanes holds the same total).
template <int V, int S = 0>
__device__ __forceinline__ void wave_halve(double (&a)[V], int lane) {
  if constexpr ((V >> S) > 1) {
    constexpr int H = (V >> S) / 2;
    const bool hi = (lane >> (5 - S)) & 1;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = hi ? a[i + H] : a[i];
      const double send = hi ? a[i] : a[i + H];
      a[i] = keep + __shfl_xor(send, 32 >> S, 64);
    }
    wave_halve<V, S + 1>(a, lane);
  }
}

__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int V>
__device__ __forceinline__ double wave_sum_multi(double (&a)[V], int lane) {
  static_assert((V & (V - 1)) == 0 && V >= 1 && V <= 64, "V: a power of two up to 64");
  wave_halve<V>(a, lane);
  double v = a[0];
#pragma unroll
  for (int off = 32 >> ilog2(V); off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__host__ __device__ constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Multi-dot body: for the columns c = wave, wave + 2 NW, ... (and c + NW
// beside each; four columns per pass when the rows fit one round) of Au/Al,
// the sums over rows [i0, i1) of
// Au[i,c] Xu[i,q] + Al[i,c] Xl[i,q] (Al, Xl may be null), reduced over the
// wave; lane 0 calls put(c, q, value).  DOT_U rows per lane per round, every
// load of a round issued before the first product.  The X columns q >= nq1
// come from a second block (Xu2, Xl2, same leading dimension) as its columns
// q - nq1; nq1 = NQ: one block.
constexpr int DOT_U = 4;

template <int NQ, int NW, class Put>
__device__ __forceinline__ void dots_body(int64_t i0, int64_t i1, int nc, const double* __restrict__ Au,
                                          const double* __restrict__ Al, int64_t lda,
                                          const double* __restrict__ Xu1, const double* __restrict__ Xl1,
                                          int64_t ldx, int nq1, const double* __restrict__ Xu2,
                                          const double* __restrict__ Xl2, int lane, int wave, Put put) {
  const double* Xu[NQ];
  const double* Xl[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    Xu[q] = q < nq1 ? Xu1 + (int64_t)q * ldx : Xu2 + (int64_t)(q - nq1) * ldx;
    Xl[q] = Xl1 == nullptr ? nullptr : q < nq1 ? Xl1 + (int64_t)q * ldx : Xl2 + (int64_t)(q - nq1) * ldx;
  }
  if (i1 - i0 <= 64 * DOT_U) {
    // the rows fit one round: the X rows stay in registers and a wave takes
    // four columns per pass (c, c + NW, c + 2 NW, c + 3 NW), every load of a
    // pass issued before its first product; the sums are formed in the same
    // order as below
    double xu[DOT_U][NQ], xl[DOT_U][NQ];
    bool in[DOT_U];
#pragma unroll
    for (int e = 0; e < DOT_U; ++e) {
      const int64_t i = i0 + e * 64 + lane;
      in[e] = i < i1;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        xu[e][q] = in[e] ? Xu[q][i] : 0.0;
        xl[e][q] = (in[e] && Xl[q]) ? Xl[q][i] : 0.0;
      }
    }
    for (int c = wave; c < nc; c += 4 * NW) {
      double u[4][DOT_U], l[4][DOT_U];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int cm = min(c + m * NW, nc - 1);   // past the end: a repeat, not stored
        const double* au = Au + (int64_t)cm * lda;
        const double* al = Al ? Al + (int64_t)cm * lda : nullptr;
#pragma unroll
        for (int e = 0; e < DOT_U; ++e) {
          const int64_t i = i0 + e * 64 + lane;
          u[m][e] = in[e] ? au[i] : 0.0;
          l[m][e] = (in[e] && al) ? al[i] : 0.0;
        }
      }
      double acc[4][NQ];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          double a = 0.0;
#pragma unroll
          for (int e = 0; e < DOT_U; ++e) a += u[m][e] * xu[e][q] + l[m][e] * xl[e][q];
          acc[m][q] = a;
        }
      constexpr int V = pow2_at_least(4 * NQ), L = ilog2(V);
      double flat[V];
#pragma unroll
      for (int t = 0; t < V; ++t) flat[t] = t < 4 * NQ ? acc[t / NQ][t % NQ] : 0.0;
      const double v = wave_sum_multi<V>(flat, lane);
      const int idx = lane >> (6 - L);
      if ((lane & ((1 << (6 - L)) - 1)) == 0 && idx < 4 * NQ && c + (idx / NQ) * NW < nc)
        put(c + (idx / NQ) * NW, idx % NQ, v);
    }
    return;
  }
  for (int c = wave; c < nc; c += 2 * NW) {
    const int c2 = c + NW;
    const bool two = c2 < nc;
    double acc[NQ], acc2[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { acc[q] = 0.0; acc2[q] = 0.0; }
    const double* au = Au + (int64_t)c * lda;
    const double* al = Al ? Al + (int64_t)c * lda : nullptr;
    const double* bu = Au + (int64_t)(two ? c2 : c) * lda;
    const double* bl = Al ? Al + (int64_t)(two ? c2 : c) * lda : nullptr;
    for (int64_t i0r = i0; i0r < i1; i0r += 64 * DOT_U) {
      double u[DOT_U], u2[DOT_U], l[DOT_U], l2[DOT_U], xu[DOT_U][NQ], xl[DOT_U][NQ];
#pragma unroll
      for (int e = 0; e < DOT_U; ++e) {
        const int64_t i = i0r + e * 64 + lane;
        const bool in = i < i1;
        u[e] = in ? au[i] : 0.0;
        u2[e] = in ? bu[i] : 0.0;
        l[e] = (in && al) ? al[i] : 0.0;
        l2[e] = (in && bl) ? bl[i] : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          xu[e][q] = in ? Xu[q][i] : 0.0;
          xl[e][q] = (in && Xl[q]) ? Xl[q][i] : 0.0;
        }
      }
#pragma unroll
      for (int e = 0; e < DOT_U; ++e)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          acc[q] += u[e] * xu[e][q] + l[e] * xl[e][q];
          acc2[q] += u2[e] * xu[e][q] + l2[e] * xl[e][q];
        }
    }
    constexpr int V = pow2_at_least(2 * NQ), L = ilog2(V);
    double flat[V];
#pragma unroll
    for (int t = 0; t < V; ++t) flat[t] = t < NQ ? acc[t] : t < 2 * NQ ? acc2[t - NQ] : 0.0;
    const double v = wave_sum_multi<V>(flat, lane);
    const int idx = lane >> (6 - L);
    if ((lane & ((1 << (6 - L)) - 1)) == 0 && idx < 2 * NQ && (idx < NQ || two))
      put(idx < NQ ? c : c2, idx % NQ, v);
  }
}

// Gram--Schmidt update of row i: Zm[i, q] -= sum_c Am[i, c] hs[c * NQ + q]
// for m = 0, 1, 2 (A1/Z1 and A2/Z2 may be null), columns in increasing order,
// UPD_U columns per round with all their loads in flight together; the
// updated rows are also left in z0, z1, z2.
constexpr int UPD_U = 8;

template <int NQ>
__device__ __forceinline__ void cgs_update_row(int64_t i, int nc, const double* hs, const double* __restrict__ A0,
                                               double* __restrict__ Z0, const double* __restrict__ A1,
                                               double* __restrict__ Z1, const double* __restrict__ A2,
                                               double* __restrict__ Z2, int64_t lda, int64_t ldz,
                                               double (&z0)[NQ], double (&z1)[NQ], double (&z2)[NQ]) {
  const bool has1 = A1 != nullptr, has2 = A2 != nullptr;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    z0[q] = Z0[i + q * ldz];
    z1[q] = has1 ? Z1[i + q * ldz] : 0.0;
    z2[q] = has2 ? Z2[i + q * ldz] : 0.0;
  }
  for (int c0 = 0; c0 < nc; c0 += UPD_U) {
    double a0[UPD_U], a1[UPD_U], a2[UPD_U];
#pragma unroll
    for (int e = 0; e < UPD_U; ++e) {
      const bool in = c0 + e < nc;
      const int64_t o = i + (int64_t)(c0 + e) * lda;
      a0[e] = in ? A0[o] : 0.0;
      a1[e] = (in && has1) ? A1[o] : 0.0;
      a2[e] = (in && has2) ? A2[o] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < UPD_U; ++e) {
      if (c0 + e >= nc) break;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double hv = hs[(c0 + e) * NQ + q];
        z0[q] -= a0[e] * hv;
        z1[q] -= a1[e] * hv;
        z2[q] -= a2[e] * hv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    Z0[i + q * ldz] = z0[q];
    if (has1) Z1[i + q * ldz] = z1[q];
    if (has2) Z2[i + q * ldz] = z2[q];
  }
}

// Gram--Schmidt tiles over 64 rows (lane = row).  Wave w owns the basis
// columns [c0, c0 + CPW) and keeps the tile's entries of Vu, Wl (and Vl) in
// registers, so that one read of the basis serves both the update z -= V h
// and the B-inner products of the updated z.
//
// Products alone (cgs_tile_dots): acc[j][q] += Vu[r, c] Xu[r, q] + Wl[r, c] Xl[r, q].
template <int NQ, int CPW>
__device__ __forceinline__ void cgs_tile_dots(int64_t r0, int64_t r1, int nc, int c0,
                                              const double* __restrict__ Vu, const double* __restrict__ Wl,
                                              int64_t lda, const double* __restrict__ Xu,
                                              const double* __restrict__ Xl, int64_t ldx, int lane,
                                              double (&acc)[CPW][NQ]) {
  const int64_t r = r0 + lane;
  const bool in = r < r1;
  const int64_t rr = in ? r : r1 - 1;   // past-the-end lanes load a valid row, contribute zero
  double au[CPW], aw[CPW], xu[NQ], xl[NQ];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int64_t o = rr + (int64_t)min(c0 + j, nc - 1) * lda;
    au[j] = Vu[o];
    aw[j] = Wl[o];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    xu[q] = in ? Xu[rr + q * ldx] : 0.0;
    xl[q] = in ? Xl[rr + q * ldx] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] += au[j] * xu[q] + aw[j] * xl[q];
}

// Update with the products (cgs_tile_update): a workgroup of NW waves owns
// NW CPW columns; z = Z - V h for (Vu, Zu), (Vl, Zl), (Wl, Zw) is stored, then
// acc[j][q] += Vu[r, c] zu[q] + Wl[r, c] zl[q].  hs: h[c NQ + q] in shared
// memory, zero from c = nc up to NW CPW.  red (NW 3 NQ 64 doubles) holds the
// waves' partial products; wave t mod NW sums column t of the block (Z minus
// the waves' parts in wave order, each part summed over its columns in
// increasing order), stores it and leaves it in fin (3 NQ 64 doubles).  Every
// wave of the workgroup calls this for every tile.
template <int NQ, int NW, int CPW>
__device__ __forceinline__ void cgs_tile_update(int64_t r0, int64_t r1, int nc, const double* hs,
                                                const double* __restrict__ Vu, const double* __restrict__ Vl,
                                                const double* __restrict__ Wl, int64_t lda, double* __restrict__ Zu,
                                                double* __restrict__ Zl, double* __restrict__ Zw, int64_t ldz,
                                                double* red, double* fin, int lane, int wave,
                                                double (&acc)[CPW][NQ]) {
  constexpr int NS = 3 * NQ;              // updated columns of the block: u, l, w parts
  constexpr int OWN = (NS + NW - 1) / NW; // block columns summed by one wave
  const int64_t r = r0 + lane;
  const bool in = r < r1;
  const int64_t rr = in ? r : r1 - 1;     // past-the-end lanes load a valid row, contribute zero
  const int c0 = wave * CPW;
  const bool has = c0 < nc;               // uniform over the wave
  double au[CPW], aw[CPW], al[CPW];
  if (has) {
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int64_t o = rr + (int64_t)min(c0 + j, nc - 1) * lda;
      au[j] = Vu[o];
      aw[j] = Wl[o];
      al[j] = Vl[o];
    }
  }
  // this wave's block columns, requested with the basis
  double zo[OWN];
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int t = wave + i * NW;
    const double* Z = t < NQ ? Zu : (t < 2 * NQ ? Zl : Zw);
    zo[i] = t < NS ? Z[rr + (t % NQ) * ldz] : 0.0;
  }
  double p[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) p[t] = 0.0;
  if (has) {
#pragma unroll
    for (int j = 0; j < CPW; ++j)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double hv = hs[(c0 + j) * NQ + q];
        p[q] += au[j] * hv;
        p[NQ + q] += al[j] * hv;
        p[2 * NQ + q] += aw[j] * hv;
      }
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) red[(wave * NS + t) * 64 + lane] = p[t];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int t = wave + i * NW;
    if (t < NS) {
      double v = zo[i];
#pragma unroll
      for (int w = 0; w < NW; ++w) v -= red[(w * NS + t) * 64 + lane];
      double* Z = t < NQ ? Zu : (t < 2 * NQ ? Zl : Zw);
      if (in) Z[rr + (t % NQ) * ldz] = v;
      fin[t * 64 + lane] = in ? v : 0.0;
    }
  }
  __syncthreads();
  if (!has) return;
  double zu[NQ], zl[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    zu[q] = fin[q * 64 + lane];
    zl[q] = fin[(NQ + q) * 64 + lane];
  }
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] += au[j] * zu[q] + aw[j] * zl[q];
}

// Sum over the wave of every lane's v (lane 0 holds the result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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
  if (bad && flag) *flag = 1;
}

constexpr int GEMM_COLS = 64;     // columns of Q staged in LDS at a time
constexpr int GEMM_KCH = 8;       // k-steps of In held in registers at a time

// LDS doubles gemm_rows_mfma needs for a given kin.
__host__ __device__ inline int gemm_lds_doubles(int kin) { return GEMM_COLS * ((kin + 3) / 4 * 4 + 1); }

// Rows [r0, r1) of Out = In * Q (In with leading dimension ldi and kin
// columns, Q kin x kout column-major, Out with leading dimension ldo), at most
// 16 * NWAVES * SLABS rows.  A dense contraction of depth kin: v_mfma_f64_16x16x4_f64,
// each wave owning SLABS slabs of 16 rows and every output column, 64 columns
// of Q at a time in LDS (column stride kin rounded up to 4, plus 1).  The In
// values of GEMM_KCH k-steps are loaded (unconditionally, from clamped
// addresses, and masked) before their products.  Called by every thread of a
// block of NWAVES waves; qs: gemm_lds_doubles(kin) doubles of shared memory.
template <int NWAVES, int SLABS>
__device__ inline void gemm_rows_mfma(int64_t r0, int64_t r1, const double* __restrict__ In, int64_t ldi, int kin,
                                      const double* __restrict__ Q, int kout, double* __restrict__ Out,
                                      int64_t ldo, double* qs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = mfma_ab_k(lane), cl = mfma_a_row(lane);   // A row = B column = lane & 15
  const int ksteps = (kin + 3) / 4, kp = ksteps * 4 + 1;
  for (int c0 = 0; c0 < kout; c0 += GEMM_COLS) {
    const int nc = min(GEMM_COLS, kout - c0);
    const int nj = (nc + 15) / 16;
    __syncthreads();   // the previous columns of Q have been consumed
    for (int idx = threadIdx.x; idx < nj * 16 * kp; idx += NWAVES * 64) {
      const int c = idx / kp, t = idx - c * kp;
      qs[idx] = (c < nc && t < kin) ? Q[(int64_t)(c0 + c) * kin + t] : 0.0;
    }
    __syncthreads();
    for (int sl = 0; sl < SLABS; ++sl) {
      const int64_t rb = r0 + (int64_t)(wave * SLABS + sl) * 16;
      if (rb >= r1) break;
      const int64_t ra = min(rb + mfma_a_row(lane), r1 - 1);
      const bool rok = rb + mfma_a_row(lane) < r1;
      dvec4 acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = dvec4{0.0, 0.0, 0.0, 0.0};
      for (int s0 = 0; s0 < ksteps; s0 += GEMM_KCH) {
        double a[GEMM_KCH];
#pragma unroll
        for (int e = 0; e < GEMM_KCH; ++e) {
          const int t = (s0 + e) * 4 + kr;
          const double v = In[ra + (int64_t)min(t, kin - 1) * ldi];
          a[e] = (rok && t < kin) ? v : 0.0;
        }
#pragma unroll
        for (int e = 0; e < GEMM_KCH; ++e) {
          if (s0 + e >= ksteps) break;
          const double* qk = qs + (s0 + e) * 4 + kr;
#pragma unroll
          // the transposed product Out^T = Q^T In^T: Q's columns are the rows
          // of the A operand, the slab's rows the columns of B, so a lane's
          // accumulator holds one output row and 16 consecutive rows are
          // stored together
          for (int j = 0; j < 4; ++j)
            if (j < nj) acc[j] = Mfma<double>::mma(qk[(j * 16 + cl) * kp], a[e], acc[j]);
        }
      }
      const int64_t row = rb + mfma_d_col(lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= nj || row >= r1) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = j * 16 + Mfma<double>::drow(lane, v);
          if (c < nc) Out[row + (int64_t)(c0 + c) * ldo] = acc[j][v];
        }
      }
    }
  }
}


// Narrow outputs (the batched form's short bases): rows [r0, r0 + rows) of
// Out = In * Q (rows <= 64, column-major Out with leading dimension ldo) with
// the In tile staged in LDS ([t][row]: the lanes of a wave read consecutive
// words) and 16 columns of Q at a time (read as broadcasts); lane = row, each
// of the 4 waves takes four of those columns.  shm: kin * 80 doubles.  Called
// by every thread of a 256-thread block.
__device__ inline void gemm_tile64(int64_t r0, int rows, const double* __restrict__ In, int64_t ldi, int kin,
                                   const double* __restrict__ Q, int kout, double* __restrict__ Out, int64_t ldo,
                                   double* shm) {
  double* tile = shm;                 // [t][row]
  double* qs = shm + (size_t)kin * 64;  // [c][t], 16 columns
  __syncthreads();   // the previous tile has been consumed
  for (int idx = threadIdx.x; idx < 64 * kin; idx += 256) {
    const int r = idx % 64, t = idx / 64;
    tile[idx] = (r < rows) ? In[r0 + r + (int64_t)t * ldi] : 0.0;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int p0 = 0; p0 < kout; p0 += 16) {
    const int np = min(16, kout - p0);
    if (p0 > 0) __syncthreads();   // the previous columns of Q have been consumed
    for (int idx = threadIdx.x; idx < 16 * kin; idx += 256) {
      const int c = idx / kin, t = idx % kin;
      qs[idx] = (c < np) ? Q[(int64_t)(p0 + c) * kin + t] : 0.0;
    }
    __syncthreads();
    const int c0 = wave * 4;
    if (c0 >= np) continue;
    const double* q = qs + (size_t)c0 * kin;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < kin; ++t) {
      const double a = tile[t * 64 + lane];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += a * q[u * kin + t];
    }
    if (lane < rows)
      for (int u = 0; u < min(4, np - c0); ++u) Out[r0 + lane + (int64_t)(p0 + c0 + u) * ldo] = acc[u];
  }
}

}  // namespace riga
