// Two-level orthogonal Arnoldi (TOAR) kernels: the Krylov basis of the
// companion pencil (eq. Linearization) kept in compact form
//   V = [U Q1; U Q2],   U: N x r with orthonormal columns,   Q = [Q1; Q2]: 2r x k,
// which the structure of the shift-and-invert operator allows: in eq.
// BlockOperatorVector the lower block of S v is r_l = sigma r_u + v_u, so the
// upper and lower blocks of every Krylov vector lie in the span of the upper
// blocks computed so far plus the start block (the compact representation of
// the second-order Arnoldi methods cited in Sec. 4.2.1; Sec. 5.2.4 notes that
// the vector work grows to rival the matrix work for large N_ev).
// Per block step only U (one N x r array) is read by the long-vector work:
// the Euclidean Gram--Schmidt of the new upper block r_u against U; the
// orthogonalisation of the Krylov block itself runs on the 2r-long compact
// coordinates in one workgroup (k_toar_compact).
#include "kernels.hpp"
#include "krylov_dev.hpp"

#include <algorithm>

namespace riga {

// ---------------------------------------------------------------------------
// One 64-row tile (lane = row) of the update Z -= U h fused with the products
// U^T Z of the updated block: wave w keeps the tile's entries of U's columns
// [w CPW, (w + 1) CPW) in registers, so one read of U serves both.  hs:
// h[c NQ + q] in LDS, zero from c = nc up to NW CPW; red: NW NQ 64 doubles,
// fin: NQ 64 doubles of LDS.  Every wave of the workgroup calls this for
// every tile.
template <int NQ, int NW, int CPW>
__device__ __forceinline__ void toar_tile(int64_t r0, int64_t r1, int nc, const double* hs,
                                          const double* __restrict__ U, int64_t ldu, double* __restrict__ Z,
                                          int64_t ldz, double* red, double* fin, int lane, int wave,
                                          double (&acc)[CPW][NQ]) {
  constexpr int OWN = (NQ + NW - 1) / NW;  // block columns summed by one wave
  const int64_t r = r0 + lane;
  const bool in = r < r1;
  const int64_t rr = in ? r : r1 - 1;      // past-the-end lanes load a valid row, contribute zero
  const int c0 = wave * CPW;
  const bool has = c0 < nc;                // uniform over the wave
  double au[CPW];
  if (has) {
#pragma unroll
    for (int j = 0; j < CPW; ++j) au[j] = U[rr + (int64_t)min(c0 + j, nc - 1) * ldu];
  }
  double zo[OWN];
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int t = wave + i * NW;
    zo[i] = t < NQ ? Z[rr + (int64_t)t * ldz] : 0.0;
  }
  double p[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) p[q] = 0.0;
  if (has) {
#pragma unroll
    for (int j = 0; j < CPW; ++j)
#pragma unroll
      for (int q = 0; q < NQ; ++q) p[q] += au[j] * hs[(c0 + j) * NQ + q];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[(wave * NQ + q) * 64 + lane] = p[q];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int t = wave + i * NW;
    if (t < NQ) {
      double v = zo[i];
#pragma unroll
      for (int w = 0; w < NW; ++w) v -= red[(w * NQ + t) * 64 + lane];
      if (in) Z[rr + (int64_t)t * ldz] = v;
      fin[t * 64 + lane] = in ? v : 0.0;
    }
  }
  __syncthreads();
  if (!has) return;
  double z[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) z[q] = fin[q * 64 + lane];
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] += au[j] * z[q];
}

// Each workgroup takes every gridDim.x-th tile and leaves one partial sum per
// output (c, q) in partial[(c NQ + q) nblk + block] for k_dots_final.
template <int NQ, int NW, int CPW>
__global__ __launch_bounds__(NW * 64) void k_toar_upd_dots(int64_t n, int nc, const double* __restrict__ h,
                                                           const double* __restrict__ U, int64_t ldu,
                                                           double* __restrict__ Z, int64_t ldz,
                                                           double* __restrict__ partial) {
  __shared__ double hs[NW * CPW * NQ];
  __shared__ double red[NW * NQ * 64];
  __shared__ double fin[NQ * 64];
  for (int k = threadIdx.x; k < NW * CPW * NQ; k += NW * 64) hs[k] = k < nc * NQ ? h[k] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[CPW][NQ];
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] = 0.0;
  const int64_t ntiles = (n + 63) / 64;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * 64;
    toar_tile<NQ, NW, CPW>(r0, min(n, r0 + 64), nc, hs, U, ldu, Z, ldz, red, fin, lane, wave, acc);
  }
  const int nblk = gridDim.x, blk = blockIdx.x;
  const int c0 = wave * CPW;
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v = acc[j][q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0 && c0 + j < nc) partial[((int64_t)(c0 + j) * NQ + q) * nblk + blk] = v;
    }
}

// Shapes: 4 waves x 8 columns (nc <= 32, nq <= 4), 8 x 12 (nc <= 96) and
// 16 x 12 (nc <= 192) for nq <= 2 (the register budget of the block columns).
constexpr int TOAR_MAX_BLOCKS = 256;   // one workgroup per compute unit

bool toar_tile_fits(int nc, int nq) {
  return nc > 0 && nq >= 1 && nq <= 4 && (nc <= 32 || (nq <= 2 && nc <= 192));
}

template <int NQ>
void launch_toar_upd_dots_nq(int blocks, int64_t n, int nc, const double* h, const double* U, int64_t ldu,
                             double* Z, int64_t ldz, double* partial, hipStream_t st) {
  if (nc <= 32) {
    hipLaunchKernelGGL((k_toar_upd_dots<NQ, 4, 8>), dim3(blocks), dim3(4 * 64), 0, st, n, nc, h, U, ldu, Z, ldz,
                       partial);
    return;
  }
  if constexpr (NQ <= 2) {
    if (nc <= 96)
      hipLaunchKernelGGL((k_toar_upd_dots<NQ, 8, 12>), dim3(blocks), dim3(8 * 64), 0, st, n, nc, h, U, ldu, Z,
                         ldz, partial);
    else
      hipLaunchKernelGGL((k_toar_upd_dots<NQ, 16, 12>), dim3(blocks), dim3(16 * 64), 0, st, n, nc, h, U, ldu, Z,
                         ldz, partial);
  }
}

int launch_toar_update_dots(int64_t n, int nc, int nq, const double* h, const double* U, int64_t ldu, double* Z,
                            int64_t ldz, double* partial, double* out, hipStream_t st) {
  if (!toar_tile_fits(nc, nq) || n <= 0) return -1;
  const int64_t ntiles = (n + 63) / 64;
  const int64_t per = (ntiles + TOAR_MAX_BLOCKS - 1) / TOAR_MAX_BLOCKS;
  const int blocks = (int)((ntiles + per - 1) / per);
  switch (nq) {
    case 1: launch_toar_upd_dots_nq<1>(blocks, n, nc, h, U, ldu, Z, ldz, partial, st); break;
    case 2: launch_toar_upd_dots_nq<2>(blocks, n, nc, h, U, ldu, Z, ldz, partial, st); break;
    case 3: launch_toar_upd_dots_nq<3>(blocks, n, nc, h, U, ldu, Z, ldz, partial, st); break;
    default: launch_toar_upd_dots_nq<4>(blocks, n, nc, h, U, ldu, Z, ldz, partial, st); break;
  }
  launch_dots_final(nc * nq, blocks, partial, out, st);
  return blocks;
}

// ---------------------------------------------------------------------------
// Compact step (one workgroup).  After the Euclidean orthonormalisation of
// the new upper block, r_u = U' [s; T] with U' = [U, u_new] (S holds s in rows
// 0..r and T in rows r..r+NQ, column q at S + q lds).  The operator's image of
// the basis block at columns k..k+NQ, whose upper coordinates are
// Q1[0:r, k:k+NQ], is then
//   x_u = [s; T],   x_l = sig x_u + [Q1[0:r, k:k+NQ]; 0]      (length r + NQ).
// x is orthogonalised against the kc = k + NQ basis columns of Q (classical
// Gram--Schmidt twice, Euclidean), H[0:kc, k+q] = h_1 + h_2,
// H[kc+c, k+q] = R[c][q] with x^T x = R^T R, and the new basis columns
// Q[:, kc+q] = (x R^{-1})[:, q] (rows r + NQ .. ldq zeroed).  P receives the new
// columns packed as [Q1 block | Q2 block] ((r + NQ) x 2NQ, column-major), the
// coefficients of the next operator input U' P.  A column whose squared norm
// after projection falls below 1e-24 of its norm before sets *flag = 1.
constexpr int TC_THREADS = 512;
constexpr int TC_MAXR = 264;   // r + NQ
constexpr int TC_MAXC = 260;   // kc
constexpr int TC_G = 8;        // lanes per basis column in the products
constexpr int TC_CH = 4;       // column chunks in the update
constexpr int TC_RT = TC_THREADS / TC_CH;   // rows per update round

template <int NQ>
__global__ __launch_bounds__(TC_THREADS) void k_toar_compact(int r, int k, double sig, const double* __restrict__ S,
                                                             int lds, double* __restrict__ Q1,
                                                             double* __restrict__ Q2, int ldq,
                                                             double* __restrict__ H, int ldh,
                                                             int* __restrict__ flag, double* __restrict__ P) {
  constexpr int NWV = TC_THREADS / 64;
  __shared__ double xu[TC_MAXR * NQ], xl[TC_MAXR * NQ];
  __shared__ double hsum[TC_MAXC * NQ], hcur[TC_MAXC * NQ];
  __shared__ double part[(TC_CH - 1) * TC_RT * 2 * NQ];   // update partial sums of chunks 1..
  __shared__ double g[NQ * NQ], hn[NQ], rinv[NQ * NQ];
  const int R2 = r + NQ, kc = k + NQ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < R2; i += TC_THREADS)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double u = S[i + q * lds];
      xu[i * NQ + q] = u;
      xl[i * NQ + q] = sig * u + (i < r ? Q1[i + (int64_t)(k + q) * ldq] : 0.0);
    }
  for (int c = tid; c < kc * NQ; c += TC_THREADS) hsum[c] = 0.0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    // h = Q^T x: TC_G consecutive lanes per basis column, rows strided by TC_G
    {
      const int grp = tid / TC_G, gl = tid % TC_G;
      for (int c = grp; c < kc; c += TC_THREADS / TC_G) {
        const double* a1 = Q1 + (int64_t)c * ldq;
        const double* a2 = Q2 + (int64_t)c * ldq;
        double p[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) p[q] = 0.0;
#pragma unroll 4
        for (int i = gl; i < R2; i += TC_G) {
          const double v1 = a1[i], v2 = a2[i];
#pragma unroll
          for (int q = 0; q < NQ; ++q) p[q] += v1 * xu[i * NQ + q] + v2 * xl[i * NQ + q];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
          for (int off = TC_G / 2; off > 0; off >>= 1) p[q] += __shfl_xor(p[q], off, 64);
          if (gl == 0) {
            hcur[c * NQ + q] = p[q];
            hsum[c * NQ + q] += p[q];
          }
        }
      }
    }
    __syncthreads();
    // x -= Q h: thread (row, chunk) sums the chunk's columns c = chunk mod TC_CH,
    // chunks 1.. leave their sums in LDS for chunk 0
    {
      const int ri = tid % TC_RT, ch = tid / TC_RT;
      for (int i0 = 0; i0 < R2; i0 += TC_RT) {
        const int i = i0 + ri;
        double su[NQ], sl[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) { su[q] = 0.0; sl[q] = 0.0; }
        if (i < R2) {
#pragma unroll 4
          for (int c = ch; c < kc; c += TC_CH) {
            const double v1 = Q1[i + (int64_t)c * ldq], v2 = Q2[i + (int64_t)c * ldq];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              su[q] += v1 * hcur[c * NQ + q];
              sl[q] += v2 * hcur[c * NQ + q];
            }
          }
        }
        if (ch > 0) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            part[((ch - 1) * TC_RT + ri) * 2 * NQ + q] = su[q];
            part[((ch - 1) * TC_RT + ri) * 2 * NQ + NQ + q] = sl[q];
          }
        }
        __syncthreads();
        if (ch == 0 && i < R2) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            double tu = su[q], tl = sl[q];
#pragma unroll
            for (int c2 = 0; c2 < TC_CH - 1; ++c2) {
              tu += part[(c2 * TC_RT + ri) * 2 * NQ + q];
              tl += part[(c2 * TC_RT + ri) * 2 * NQ + NQ + q];
            }
            xu[i * NQ + q] -= tu;
            xl[i * NQ + q] -= tl;
          }
        }
        __syncthreads();
      }
    }
  }
  for (int idx = tid; idx < kc * NQ; idx += TC_THREADS) {
    const int c = idx / NQ, q = idx % NQ;
    H[c + (int64_t)(k + q) * ldh] = hsum[idx];
  }
  // Gram matrix of the projected block and the squared norms of the
  // coefficients (the norm before projection is their sum, by Pythagoras)
  for (int idx = wave; idx < NQ * NQ + NQ; idx += NWV) {
    double s = 0.0;
    if (idx < NQ * NQ) {
      const int a = idx / NQ, q = idx % NQ;
      for (int i = lane; i < R2; i += 64) s += xu[i * NQ + a] * xu[i * NQ + q] + xl[i * NQ + a] * xl[i * NQ + q];
    } else {
      const int q = idx - NQ * NQ;
      for (int c = lane; c < kc; c += 64) s += hsum[c * NQ + q] * hsum[c * NQ + q];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
      if (idx < NQ * NQ) g[idx] = s; else hn[idx - NQ * NQ] = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double R[NQ][NQ], X[NQ][NQ];
    bool bad = false;
    for (int a = 0; a < NQ; ++a)
      for (int q = 0; q < NQ; ++q) { R[a][q] = 0.0; X[a][q] = 0.0; }
    for (int j = 0; j < NQ; ++j) {
      const double n0 = g[j * NQ + j] + hn[j];
      for (int i = 0; i <= j; ++i) {
        double s = 0.5 * (g[i * NQ + j] + g[j * NQ + i]);
        for (int t = 0; t < i; ++t) s -= R[t][i] * R[t][j];
        if (i == j) {
          if (!(s > 1e-24 * n0)) { bad = true; s = 1.0; }
          R[j][j] = sqrt(s);
        } else {
          R[i][j] = s / R[i][i];
        }
      }
    }
    for (int j = 0; j < NQ; ++j) {
      X[j][j] = 1.0 / R[j][j];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int t = i + 1; t <= j; ++t) s += R[i][t] * X[t][j];
        X[i][j] = -s / R[i][i];
      }
    }
    for (int q = 0; q < NQ; ++q)
      for (int c = 0; c < NQ; ++c) {
        H[kc + c + (int64_t)(k + q) * ldh] = R[c][q];
        rinv[c * NQ + q] = X[c][q];
      }
    if (bad) *flag = 1;
  }
  __syncthreads();
  for (int i = tid; i < ldq; i += TC_THREADS) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v1 = 0.0, v2 = 0.0;
      if (i < R2) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          v1 += xu[i * NQ + a] * rinv[a * NQ + q];
          v2 += xl[i * NQ + a] * rinv[a * NQ + q];
        }
        P[i + q * R2] = v1;
        P[i + (NQ + q) * R2] = v2;
      }
      Q1[i + (int64_t)(kc + q) * ldq] = v1;
      Q2[i + (int64_t)(kc + q) * ldq] = v2;
    }
  }
}

bool launch_toar_compact(int r, int k, int nq, double sig, const double* S, int lds, double* Q1, double* Q2, int ldq,
                         double* H, int ldh, int* flag, double* P, hipStream_t st) {
  if (nq < 1 || nq > 4 || r + nq > TC_MAXR || k + nq > TC_MAXC || r + nq > ldq) return false;
#define RIGA_TC(NQ)                                                                                        \
  hipLaunchKernelGGL(k_toar_compact<NQ>, dim3(1), dim3(TC_THREADS), 0, st, r, k, sig, S, lds, Q1, Q2, ldq, H, \
                     ldh, flag, P)
  switch (nq) {
    case 1: RIGA_TC(1); break;
    case 2: RIGA_TC(2); break;
    case 3: RIGA_TC(3); break;
    default: RIGA_TC(4); break;
  }
#undef RIGA_TC
  return true;
}

}  // namespace riga
