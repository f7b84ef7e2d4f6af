// Building blocks of the Krylov iteration (Alg. 2): sparse products with the
// assembled matrices (lines 8-11), B-inner products and Gram--Schmidt updates
// (lines 9-12), and tall-skinny products for restarts and Ritz vectors.
// All of these are HBM-bound: rows are the long dimension, columns (Krylov
// vectors) the short one, and every kernel streams each matrix or basis column
// once with coalesced accesses.
#include "kernels.hpp"
#include "krylov_dev.hpp"

#include <algorithm>

namespace riga {

// ---------------------------------------------------------------------------
// SpMV with the implicit tensor sparsity: row (i, j) couples to columns
// (ii, jj) with ii in [lo(i), hi(i)], jj in [lo(j), hi(j)], stored row-major
// in that order, so no column-index array is read.  16 lanes per row.
constexpr int SPMV_THREADS = 256;

template <int NC>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv(
    int n, const int* __restrict__ lo, const int* __restrict__ hi, const int64_t* __restrict__ rowptr,
    int64_t ndof, const double* __restrict__ A, double a, const double* __restrict__ X, int64_t ldx,
    double* __restrict__ Y, int64_t ldy, const double* __restrict__ Z, int64_t ldz, double bz,
    double* __restrict__ Y2, int64_t ldy2) {
  const int g = threadIdx.x % SPMV_G;
  const int64_t r = ((int64_t)blockIdx.x * SPMV_THREADS + threadIdx.x) / SPMV_G;
  const bool active = r < ndof;
  double s[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) s[q] = 0.0;
  if (active) {
    // rows fit in 32 bits (far more than a device holds); the index loads are
    // all issued before the first of them is used
    const unsigned ru = (unsigned)r, j = ru / (unsigned)n, i = ru - j * (unsigned)n;
    const int lx = lo[i], hx = hi[i], ly = lo[j];
    const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
    asm volatile("" ::"v"(lx), "v"(hx), "v"(ly));
    tensor_row_sum<NC>(A + k0, (int)(k1 - k0), X + (int64_t)ly * n + lx, ldx, n, hx - lx + 1, g, s);
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int off = SPMV_G / 2; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, SPMV_G);
  if (active && g == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      double val = a * s[q];
      if (Z) val += bz * Z[r + q * ldz];
      Y[r + q * ldy] = val;
      if (Y2) Y2[r + q * ldy2] = s[q];
    }
  }
}

// The same product with explicit column indices (vector spaces): SPMV_G
// lanes per row, entries strided by SPMV_G.
template <int NC>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv_csr(
    const int* __restrict__ col, const int64_t* __restrict__ rowptr, int64_t ndof, const double* __restrict__ A,
    double a, const double* __restrict__ X, int64_t ldx, double* __restrict__ Y, int64_t ldy,
    const double* __restrict__ Z, int64_t ldz, double bz, double* __restrict__ Y2, int64_t ldy2) {
  const int g = threadIdx.x % SPMV_G;
  const int64_t r = ((int64_t)blockIdx.x * SPMV_THREADS + threadIdx.x) / SPMV_G;
  const bool active = r < ndof;
  double s[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) s[q] = 0.0;
  if (active) {
    const int64_t k1 = rowptr[r + 1];
    for (int64_t k = rowptr[r] + g; k < k1; k += SPMV_G) {
      const double av = A[k];
      const int64_t c = col[k];
#pragma unroll
      for (int q = 0; q < NC; ++q) s[q] += av * X[c + q * ldx];
    }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int off = SPMV_G / 2; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, SPMV_G);
  if (active && g == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      double val = a * s[q];
      if (Z) val += bz * Z[r + q * ldz];
      Y[r + q * ldy] = val;
      if (Y2) Y2[r + q * ldy2] = s[q];
    }
  }
}

void launch_spmv(const DevSpace& s, int64_t ndof, int ncols, const double* A, double a, const double* X,
                 int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz, double bz, double* Y2,
                 int64_t ldy2, hipStream_t st) {
  int64_t blocks = (ndof * SPMV_G + SPMV_THREADS - 1) / SPMV_THREADS;
  if (s.col != nullptr) {
#define RIGA_SPMVC(NC)                                                                                      \
  hipLaunchKernelGGL(k_spmv_csr<NC>, dim3((unsigned)blocks), dim3(SPMV_THREADS), 0, st, s.col, s.rowptr, ndof, A, a, \
                     X, ldx, Y, ldy, Z, ldz, bz, Y2, ldy2)
    switch (ncols) {
      case 1: RIGA_SPMVC(1); break;
      case 2: RIGA_SPMVC(2); break;
      case 3: RIGA_SPMVC(3); break;
      case 4: RIGA_SPMVC(4); break;
      case 5: RIGA_SPMVC(5); break;
      case 6: RIGA_SPMVC(6); break;
      case 7: RIGA_SPMVC(7); break;
      default: RIGA_SPMVC(8); break;
    }
#undef RIGA_SPMVC
    return;
  }
#define RIGA_SPMV(NC)                                                                              \
  hipLaunchKernelGGL(k_spmv<NC>, dim3((unsigned)blocks), dim3(SPMV_THREADS), 0, st, s.n, s.lo, s.hi, \
                     s.rowptr, ndof, A, a, X, ldx, Y, ldy, Z, ldz, bz, Y2, ldy2)
  switch (ncols) {
    case 1: RIGA_SPMV(1); break;
    case 2: RIGA_SPMV(2); break;
    case 3: RIGA_SPMV(3); break;
    case 4: RIGA_SPMV(4); break;
    case 5: RIGA_SPMV(5); break;
    case 6: RIGA_SPMV(6); break;
    case 7: RIGA_SPMV(7); break;
    default: RIGA_SPMV(8); break;
  }
#undef RIGA_SPMV
}

// ---------------------------------------------------------------------------
// Sliced-ELL products: a workgroup per slab of 64 rows, lane = row, its waves
// taking interleaved rounds of entries (partial sums added in LDS in wave
// order).  The matrix is read in 512-byte coalesced rows of the slab; the
// vector entries of a row are
// the implicit tensor columns, which consecutive rows of a grid line share
// shifted by one, so the gathers of a wave fall on a few cache lines.
int64_t build_ell_slabs(const std::vector<int64_t>& rowptr, const std::vector<int4>& ranges,
                        std::vector<EllSlab>& slabs) {
  slabs.clear();
  int64_t off = 0;
  for (const int4& rg : ranges)
    for (int64_t r = rg.y; r < rg.z; r += 64) {
      EllSlab sb{};
      sb.inst = rg.x;
      sb.r0 = (int)r;
      sb.nrows = (int)std::min<int64_t>(64, rg.z - r);
      int w = 0;
      for (int l = 0; l < sb.nrows; ++l) w = std::max(w, (int)(rowptr[r + l + 1] - rowptr[r + l]));
      sb.width = w;
      sb.off = off;
      off += (int64_t)w * 64;
      slabs.push_back(sb);
    }
  return off;
}

__global__ __launch_bounds__(64) void k_csr_to_ell(const EllSlab* __restrict__ slabs,
                                                   const int64_t* __restrict__ rowptr,
                                                   const double* __restrict__ V, double* __restrict__ E) {
  const EllSlab sb = slabs[blockIdx.x];
  const int l = threadIdx.x;
  const bool act = l < sb.nrows;
  int64_t k0 = 0, len = 0;
  if (act) {
    k0 = rowptr[sb.r0 + l];
    len = rowptr[sb.r0 + l + 1] - k0;
  }
  for (int o = 0; o < sb.width; ++o) E[sb.off + (int64_t)o * 64 + l] = (o < len) ? V[k0 + o] : 0.0;
}

void launch_csr_to_ell(const EllSlab* slabs, int nslab, const int64_t* rowptr, const double* V, double* E,
                       hipStream_t st) {
  if (nslab <= 0) return;
  hipLaunchKernelGGL(k_csr_to_ell, dim3(nslab), dim3(64), 0, st, slabs, rowptr, V, E);
}

constexpr int ELL_U = 7;   // entries per round: one stencil line of a degree-3 row
constexpr int ELL_W = 4;   // waves per slab, taking interleaved rounds

template <int NC>
__global__ __launch_bounds__(ELL_W * 64) void k_spmv_ell(const EllSlab* __restrict__ slabs, int nslab,
                                                         const DevSpace* __restrict__ spaces,
                                                         const int64_t* __restrict__ dofbase,
                                                         const unsigned char* __restrict__ live,
                                                         const double* __restrict__ E, const double* __restrict__ X,
                                                         int64_t ldx, double* __restrict__ Y, int64_t ldy,
                                                         const double* __restrict__ Z, int64_t ldz, double bz) {
  __shared__ double red[ELL_W][64][NC];
  const EllSlab sb = slabs[blockIdx.x];
  if (live != nullptr && !live[sb.inst]) return;
  const DevSpace sp = spaces[sb.inst];
  const int64_t base = dofbase != nullptr ? dofbase[sb.inst] : 0;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool act = l < sb.nrows;
  const unsigned rl = (unsigned)(sb.r0 - base) + (act ? (unsigned)l : 0u);   // row within its problem
  const unsigned n = (unsigned)sp.n, j = rl / n, i = rl - j * n;
  const int lx = sp.lo[i], hx = sp.hi[i], ly = sp.lo[j], hy = sp.hi[j];
  const int wx = hx - lx + 1, len = wx * (hy - ly + 1);
  const double* xb = X + base + (int64_t)ly * n + lx;
  const double* xr = X + base + rl;          // a valid address for padded entries
  const double* e = E + sb.off + l;
  double acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = 0.0;
  for (int o0 = w * ELL_U; o0 < sb.width; o0 += ELL_W * ELL_U) {
    double av[ELL_U], xv[ELL_U][NC];
#pragma unroll
    for (int u = 0; u < ELL_U; ++u) {
      const int o = o0 + u;
      const double a = e[(int64_t)min(o, sb.width - 1) * 64];
      av[u] = (o < sb.width) ? a : 0.0;
      const int dy = o / wx;
      const double* xp = (o < len) ? xb + (int64_t)dy * n + (o - dy * wx) : xr;
#pragma unroll
      for (int q = 0; q < NC; ++q) xv[u][q] = xp[q * ldx];
    }
#pragma unroll
    for (int u = 0; u < ELL_U; ++u)
#pragma unroll
      for (int q = 0; q < NC; ++q) acc[q] += av[u] * xv[u][q];
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) red[w][l][q] = acc[q];
  __syncthreads();
  if (w == 0 && act) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      double val = 0.0;
#pragma unroll
      for (int v = 0; v < ELL_W; ++v) val += red[v][l][q];
      if (Z) val += bz * Z[base + rl + q * ldz];
      Y[base + rl + q * ldy] = val;
    }
  }
}

void launch_spmv_ell(const EllSlab* slabs, int nslab, const DevSpace* spaces, const int64_t* dofbase,
                     const unsigned char* live, int ncols, const double* E, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, const double* Z, int64_t ldz, double bz, hipStream_t st) {
  if (nslab <= 0) return;
#define RIGA_SPMV_ELL(NC)                                                                                        \
  hipLaunchKernelGGL(k_spmv_ell<NC>, dim3(nslab), dim3(ELL_W * 64), 0, st, slabs, nslab, spaces, dofbase, live, E, X, \
                     ldx, Y, ldy, Z, ldz, bz)
  switch (ncols) {
    case 1: RIGA_SPMV_ELL(1); break;
    case 2: RIGA_SPMV_ELL(2); break;
    case 3: RIGA_SPMV_ELL(3); break;
    default: RIGA_SPMV_ELL(4); break;
  }
#undef RIGA_SPMV_ELL
}

// Three products with one pass over X: Y0 = A0 X, Y1 = A1 X, Y2 = A2 X.
template <int NC>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv3(
    int n, const int* __restrict__ lo, const int* __restrict__ hi, const int* __restrict__ colidx,
    const int64_t* __restrict__ rowptr, int64_t ndof, const double* __restrict__ A0, const double* __restrict__ A1,
    const double* __restrict__ A2, const double* __restrict__ X, int64_t ldx, double* __restrict__ Y0,
    double* __restrict__ Y1, double* __restrict__ Y2, int64_t ldy) {
  const int g = threadIdx.x % SPMV_G;
  const int64_t r = ((int64_t)blockIdx.x * SPMV_THREADS + threadIdx.x) / SPMV_G;
  const bool active = r < ndof;
  double s0[NC], s1[NC], s2[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) { s0[q] = 0.0; s1[q] = 0.0; s2[q] = 0.0; }
  if (active) {
    // explicit columns (vector spaces), else the tensor pattern of the scalar space
    int lx = 0, wx = 1, ly = 0;
    if (colidx == nullptr) {
      const unsigned ru = (unsigned)r, j = ru / (unsigned)n, i = ru - j * (unsigned)n;
      lx = lo[i]; wx = hi[i] - lo[i] + 1; ly = lo[j];
    }
    const int64_t k0 = rowptr[r], len = rowptr[r + 1] - k0;
    for (int o = g; o < len; o += SPMV_G) {
      const int64_t col = colidx != nullptr ? (int64_t)colidx[k0 + o] : (int64_t)(ly + o / wx) * n + lx + o % wx;
      const double v0 = A0[k0 + o], v1 = A1[k0 + o], v2 = A2[k0 + o];
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const double xv = X[col + q * ldx];
        s0[q] += v0 * xv;
        s1[q] += v1 * xv;
        s2[q] += v2 * xv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int off = SPMV_G / 2; off > 0; off >>= 1) {
      s0[q] += __shfl_xor(s0[q], off, SPMV_G);
      s1[q] += __shfl_xor(s1[q], off, SPMV_G);
      s2[q] += __shfl_xor(s2[q], off, SPMV_G);
    }
  if (active && g == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Y0[r + q * ldy] = s0[q];
      Y1[r + q * ldy] = s1[q];
      Y2[r + q * ldy] = s2[q];
    }
  }
}

void launch_spmv3(const DevSpace& s, int64_t ndof, int ncols, const double* A0, const double* A1, const double* A2,
                  const double* X, int64_t ldx, double* Y0, double* Y1, double* Y2, int64_t ldy, hipStream_t st) {
  int64_t blocks = (ndof * SPMV_G + SPMV_THREADS - 1) / SPMV_THREADS;
#define RIGA_SPMV3(NC)                                                                              \
  hipLaunchKernelGGL(k_spmv3<NC>, dim3((unsigned)blocks), dim3(SPMV_THREADS), 0, st, s.n, s.lo, s.hi, s.col, \
                     s.rowptr, ndof, A0, A1, A2, X, ldx, Y0, Y1, Y2, ldy)
  switch (ncols) {
    case 1: RIGA_SPMV3(1); break;
    case 2: RIGA_SPMV3(2); break;
    case 3: RIGA_SPMV3(3); break;
    case 4: RIGA_SPMV3(4); break;
    case 5: RIGA_SPMV3(5); break;
    case 6: RIGA_SPMV3(6); break;
    case 7: RIGA_SPMV3(7); break;
    default: RIGA_SPMV3(8); break;
  }
#undef RIGA_SPMV3
}

// ---------------------------------------------------------------------------
// Multi-dot products out[c][q] = sum_i Au[i,c] Xu[i,q] + Al[i,c] Xl[i,q]:
// each block owns a slice of rows, each wave owns a set of columns c and its
// lanes stride the slice (coalesced loads, two columns in flight per wave).
// Per-block partial sums are stored output-major, partial[(c*NQ+q)*nblk + blk],
// and a second kernel reduces each output with one wave (deterministic order).
constexpr int DOT_THREADS = 256;

int dots_blocks(int64_t n) {
  int64_t b = (n + 127) / 128;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

template <int NQ>
__global__ __launch_bounds__(DOT_THREADS) void k_dots(
    int64_t n, int nc, const double* __restrict__ Au, const double* __restrict__ Al, int64_t lda,
    const double* __restrict__ Xu, const double* __restrict__ Xl, int64_t ldx,
    double* __restrict__ partial) {
  const int nblk = gridDim.x;
  const int64_t per = (n + nblk - 1) / nblk;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = min(n, i0 + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = blockIdx.x;
  dots_body<NQ, DOT_THREADS / 64>(i0, i1, nc, Au, Al, lda, Xu, Xl, ldx, NQ, nullptr, nullptr, lane, wave,
                                  [&](int c, int q, double v) { partial[((int64_t)c * NQ + q) * nblk + blk] = v; });
}

__global__ __launch_bounds__(256) void k_dots_final(int nout, int nblk, const double* __restrict__ partial,
                                                    double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (idx >= nout) return;
  const double* p = partial + (int64_t)idx * nblk;
  // partials lane, lane + 64, ... in that order, eight loads in flight
  double s = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int b = b0 + e * 64 + lane;
      v[e] = b < nblk ? p[b] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) s += v[e];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[idx] = s;
}

void launch_dots_final(int nout, int nblk, const double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dots_final, dim3((nout + 3) / 4), dim3(256), 0, st, nout, nblk, partial, out);
}

void launch_dots(int64_t n, int nc, const double* Au, const double* Al, int64_t lda,
                 int nq, const double* Xu, const double* Xl, int64_t ldx,
                 double* partial, double* out, hipStream_t st) {
  if (nc <= 0) return;
  int blocks = dots_blocks(n);
#define RIGA_DOTS(NQ)                                                                          \
  hipLaunchKernelGGL(k_dots<NQ>, dim3(blocks), dim3(DOT_THREADS), 0, st, n, nc, Au, Al, lda, Xu, \
                     Xl, ldx, partial)
  switch (nq) {
    case 1: RIGA_DOTS(1); break;
    case 2: RIGA_DOTS(2); break;
    case 3: RIGA_DOTS(3); break;
    default: RIGA_DOTS(4); break;
  }
#undef RIGA_DOTS
  const int nout = nc * nq;
  hipLaunchKernelGGL(k_dots_final, dim3((nout + 3) / 4), dim3(256), 0, st, nout, blocks, partial, out);
}

// ---------------------------------------------------------------------------
// Sum-factorised products with M = M1 (x) M1 and K = K1 (x) M1 + M1 (x) K1
// (banded 1-D factors, band width w = 2p + 1, entry (i, ii) at
// i w + ii - i + p).  A workgroup owns a tile of TT_I x TT_J grid points: it
// stages X on the tile plus a halo of p in shared memory, forms
// TM = X M1^T and TK = X K1^T along i for the tile's rows and the halo rows,
// then Y = M1 (a TM + b TK) + b K1 TM along j.
constexpr int TT_I = TENSOR_TILE_I, TT_J = TENSOR_TILE_J, TT_THREADS = 256;
// Tile height of the single-problem launches: half the forest's, so a
// single grid gives twice the workgroups (these launches are latency-bound).
constexpr int TT_J1 = TENSOR_TILE_J / 2;

// One tile (i0, j0) of TT_I x TJ points of one grid; sm: shared memory for
// the halo and the partial products (sized for the largest degree of the
// launch).
template <int NQ, bool HASK, int TJ = TT_J>
__device__ __forceinline__ void tensor_tile(int n, int p, int i0, int j0, const double* __restrict__ M1,
                                            const double* __restrict__ K1, double a, double b,
                                            const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                                            int64_t ldy, const double* __restrict__ Z, int64_t ldz, double c,
                                            double* sm) {
  const int w = 2 * p + 1;
  const int hx = TT_I + 2 * p, hy = TJ + 2 * p;
  double* xs = sm;                          // [hy][hx][NQ]
  double* tm = xs + (size_t)hy * hx * NQ;   // [hy][TT_I][NQ]
  double* tk = tm + (size_t)hy * TT_I * NQ; // [hy][TT_I][NQ] (HASK)
  for (int idx = threadIdx.x; idx < hy * hx; idx += TT_THREADS) {
    const int jj = j0 - p + idx / hx, ii = i0 - p + idx % hx;
    const bool in = jj >= 0 && jj < n && ii >= 0 && ii < n;
    const int64_t d = (int64_t)jj * n + ii;
#pragma unroll
    for (int q = 0; q < NQ; ++q) xs[idx * NQ + q] = in ? X[d + q * ldx] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < hy * TT_I; idx += TT_THREADS) {
    const int r = idx / TT_I, ci = idx % TT_I, i = min(i0 + ci, n - 1);
    const double* mb = M1 + (int64_t)i * w;
    const double* kb = K1 + (int64_t)i * w;
    const double* xr = xs + ((size_t)r * hx + ci) * NQ;   // column i - p of the halo row
    double sm_[NQ], sk_[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { sm_[q] = 0.0; sk_[q] = 0.0; }
    for (int o = 0; o < w; ++o) {
      const double mv = mb[o], kv = HASK ? kb[o] : 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        sm_[q] += mv * xr[o * NQ + q];
        if (HASK) sk_[q] += kv * xr[o * NQ + q];
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      tm[idx * NQ + q] = sm_[q];
      if (HASK) tk[idx * NQ + q] = sk_[q];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TJ * TT_I; idx += TT_THREADS) {
    const int jr = idx / TT_I, ci = idx % TT_I;
    const int i = i0 + ci, j = j0 + jr;
    if (i >= n || j >= n) continue;
    const double* mb = M1 + (int64_t)j * w;
    const double* kb = K1 + (int64_t)j * w;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int o = 0; o < w; ++o) {
      const size_t t = ((size_t)(jr + o) * TT_I + ci) * NQ;   // row j - p + o of the halo
      const double mv = mb[o];
      if (HASK) {
        const double kv = kb[o], am = a * mv + b * kv, bm = b * mv;
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += am * tm[t + q] + bm * tk[t + q];
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += mv * tm[t + q];
      }
    }
    const int64_t d = (int64_t)j * n + i;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double v = HASK ? acc[q] : a * acc[q];
      if (Z) v += c * Z[d + q * ldz];
      Y[d + q * ldy] = v;
    }
  }
}

template <int NQ, bool HASK>
__global__ __launch_bounds__(TT_THREADS) void k_tensor_mk(int n, int p, const double* __restrict__ M1,
                                                          const double* __restrict__ K1, double a, double b,
                                                          const double* __restrict__ X, int64_t ldx,
                                                          double* __restrict__ Y, int64_t ldy,
                                                          const double* __restrict__ Z, int64_t ldz, double c) {
  extern __shared__ double sm[];
  tensor_tile<NQ, HASK, TT_J1>(n, p, blockIdx.x * TT_I, blockIdx.y * TT_J1, M1, K1, a, b, X, ldx, Y, ldy, Z, ldz, c,
                               sm);
}

// Every live problem of a forest: tile t = {problem, i0, j0, 0}; the problem's
// rows start at dofbase, its bands at bandoff; a = sig + alpha, b = beta, or
// with sig null a = 1, b = 0.
template <int NQ, bool HASK>
__global__ __launch_bounds__(TT_THREADS) void k_tensor_mk_b(const int4* __restrict__ tiles,
                                                            const DevSpace* __restrict__ spaces,
                                                            const int64_t* __restrict__ dofbase,
                                                            const int64_t* __restrict__ bandoff,
                                                            const double* __restrict__ M1,
                                                            const double* __restrict__ K1,
                                                            const unsigned char* __restrict__ live,
                                                            const double* __restrict__ sig,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta,
                                                            const double* __restrict__ X, int64_t ldx,
                                                            double* __restrict__ Y, int64_t ldy,
                                                            const double* __restrict__ Z, int64_t ldz, double c) {
  extern __shared__ double sm[];
  const int4 tl = tiles[blockIdx.x];
  const int q = tl.x;
  if (live != nullptr && !live[q]) return;   // the whole workgroup leaves together
  const int n = spaces[q].n, p = spaces[q].p;
  const int64_t base = dofbase[q], bo = bandoff[q];
  const double a = sig ? sig[q] + alpha[q] : 1.0, b = sig ? beta[q] : 0.0;
  tensor_tile<NQ, HASK>(n, p, tl.y, tl.z, M1 + bo, K1 + bo, a, b, X + base, ldx, Y + base, ldy,
                        Z ? Z + base : nullptr, ldz, c, sm);
}

size_t tensor_shm(int max_p, int nq, bool hask, int tj) {
  const size_t shm_x = (size_t)(tj + 2 * max_p) * (TT_I + 2 * max_p), shm_t = (size_t)(tj + 2 * max_p) * TT_I;
  return (shm_x + (hask ? 2 : 1) * shm_t) * nq * sizeof(double);
}

void launch_tensor_mk_b(const int4* tiles, int ntiles, const DevSpace* spaces, const int64_t* dofbase,
                        const int64_t* bandoff, const double* M1, const double* K1, const unsigned char* live,
                        const double* sig, const double* alpha, const double* beta, int nq, int max_p,
                        const double* X, int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz,
                        double c, hipStream_t st) {
  if (ntiles <= 0) return;
  const bool hask = sig != nullptr;
#define RIGA_TMKB(NQ)                                                                                          \
  do {                                                                                                         \
    const size_t shm = tensor_shm(max_p, NQ, hask, TT_J);                                                            \
    if (hask)                                                                                                  \
      hipLaunchKernelGGL((k_tensor_mk_b<NQ, true>), dim3(ntiles), dim3(TT_THREADS), shm, st, tiles, spaces,      \
                         dofbase, bandoff, M1, K1, live, sig, alpha, beta, X, ldx, Y, ldy, Z, ldz, c);         \
    else                                                                                                       \
      hipLaunchKernelGGL((k_tensor_mk_b<NQ, false>), dim3(ntiles), dim3(TT_THREADS), shm, st, tiles, spaces,     \
                         dofbase, bandoff, M1, K1, live, sig, alpha, beta, X, ldx, Y, ldy, Z, ldz, c);         \
  } while (0)
  switch (nq) {
    case 1: RIGA_TMKB(1); break;
    case 2: RIGA_TMKB(2); break;
    case 3: RIGA_TMKB(3); break;
    default: RIGA_TMKB(4); break;
  }
#undef RIGA_TMKB
}

void launch_tensor_mk(const DevSpace& s, const double* M1, const double* K1, int nq, double a, double b,
                      const double* X, int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz, double c,
                      hipStream_t st) {
  const int n = s.n, p = s.p;
  if (n <= 0) return;
  const dim3 grid((n + TT_I - 1) / TT_I, (n + TT_J1 - 1) / TT_J1);
  const bool hask = b != 0.0;
#define RIGA_TMK(NQ)                                                                                           \
  do {                                                                                                         \
    const size_t shm = tensor_shm(p, NQ, hask, TT_J1);                                                                \
    if (hask)                                                                                                  \
      hipLaunchKernelGGL((k_tensor_mk<NQ, true>), grid, dim3(TT_THREADS), shm, st, n, p, M1, K1, a, b, X, ldx, Y, \
                         ldy, Z, ldz, c);                                                                      \
    else                                                                                                       \
      hipLaunchKernelGGL((k_tensor_mk<NQ, false>), grid, dim3(TT_THREADS), shm, st, n, p, M1, K1, a, b, X, ldx,  \
                         Y, ldy, Z, ldz, c);                                                                   \
  } while (0)
  switch (nq) {
    case 1: RIGA_TMK(1); break;
    case 2: RIGA_TMK(2); break;
    case 3: RIGA_TMK(3); break;
    default: RIGA_TMK(4); break;
  }
#undef RIGA_TMK
}

// Pass 1 products (as launch_dots) and Y = M X (sum-factorised, as
// launch_tensor_mk with b = 0) in one launch: the first nblk workgroups form
// the products, the others the tiles of the mass product.  The two read
// different data and write different outputs.
template <int NQ>
__global__ __launch_bounds__(256) void k_dots_mr(int64_t n, int nc, const double* __restrict__ Au,
                                                 const double* __restrict__ Al, int64_t lda,
                                                 const double* __restrict__ Xu, const double* __restrict__ Xl,
                                                 int64_t ldx, double* __restrict__ partial, int nblk, int tn, int p,
                                                 const double* __restrict__ M1, const double* __restrict__ X2,
                                                 int64_t ldx2, double* __restrict__ Y2, int64_t ldy2) {
  extern __shared__ double sm[];
  const int bx = blockIdx.x;
  if (bx < nblk) {
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t i0 = (int64_t)bx * per;
    const int64_t i1 = min(n, i0 + per);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    dots_body<NQ, 4>(i0, i1, nc, Au, Al, lda, Xu, Xl, ldx, NQ, nullptr, nullptr, lane, wave,
                     [&](int c, int q, double v) { partial[((int64_t)c * NQ + q) * nblk + bx] = v; });
  } else {
    const int t = bx - nblk, gx = (tn + TT_I - 1) / TT_I;
    tensor_tile<NQ, false, TT_J1>(tn, p, (t % gx) * TT_I, (t / gx) * TT_J1, M1, nullptr, 1.0, 0.0, X2, ldx2, Y2, ldy2,
                           nullptr, 0, 0.0, sm);
  }
}

void launch_dots_mr(int64_t n, int nc, const double* Au, const double* Al, int64_t lda, int nq, const double* Xu,
                    const double* Xl, int64_t ldx, double* partial, double* out, const DevSpace& s,
                    const double* M1, double* Y2, int64_t ldy2, hipStream_t st) {
  const int blocks = dots_blocks(n);
  const int tn = s.n, gx = (tn + TT_I - 1) / TT_I, gy = (tn + TT_J1 - 1) / TT_J1;
  const unsigned grid = (unsigned)(blocks + gx * gy);
  const size_t shm = tensor_shm(s.p, nq, false, TT_J1);
#define RIGA_DMR(NQ)                                                                                        \
  hipLaunchKernelGGL(k_dots_mr<NQ>, dim3(grid), dim3(256), shm, st, n, nc, Au, Al, lda, Xu, Xl, ldx, partial, \
                     blocks, tn, s.p, M1, Xl, ldx, Y2, ldy2)
  switch (nq) {
    case 1: RIGA_DMR(1); break;
    case 2: RIGA_DMR(2); break;
    case 3: RIGA_DMR(3); break;
    default: RIGA_DMR(4); break;
  }
#undef RIGA_DMR
  const int nout = nc * nq;
  hipLaunchKernelGGL(k_dots_final, dim3((nout + 3) / 4), dim3(256), 0, st, nout, blocks, partial, out);
}

// ---------------------------------------------------------------------------
// Gram--Schmidt update Z[:, q] -= sum_c A[:, c] h[c][q] for up to three
// (A, Z) pairs sharing h (upper part, lower part, and M times the lower part).
constexpr int UPD_THREADS = 256;

template <int NQ>
__global__ __launch_bounds__(UPD_THREADS) void k_cgs_update(
    int64_t n, int nc, const double* __restrict__ h,
    const double* __restrict__ A0, double* __restrict__ Z0, const double* __restrict__ A1,
    double* __restrict__ Z1, const double* __restrict__ A2, double* __restrict__ Z2,
    int64_t lda, int64_t ldz, double* __restrict__ gpart) {
  extern __shared__ double hs[];
  for (int k = threadIdx.x; k < nc * NQ; k += UPD_THREADS) hs[k] = h[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x;
  double z0[NQ], z1[NQ], z2[NQ];
  if (i < n) cgs_update_row<NQ>(i, nc, hs, A0, Z0, A1, Z1, A2, Z2, lda, ldz, z0, z1, z2);
  if (gpart == nullptr) return;
  // B-Gram of the updated block, Z0^T Z0 + Z2^T Z1 (Z2 = M Z1), summed over
  // the block's rows: lanes, then waves in order
  __shared__ double gw[UPD_THREADS / 64][NQ * NQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NQ; ++c)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double g = (i < n) ? z0[c] * z0[q] + z2[c] * z1[q] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off, 64);
      if (lane == 0) gw[wave][c * NQ + q] = g;
    }
  __syncthreads();
  if (threadIdx.x < NQ * NQ) {
    double g = 0.0;
#pragma unroll
    for (int w = 0; w < UPD_THREADS / 64; ++w) g += gw[w][threadIdx.x];
    gpart[(int64_t)blockIdx.x * NQ * NQ + threadIdx.x] = g;
  }
}

int launch_cgs_update(int64_t n, int nc, int nq, const double* h,
                      const double* A0, double* Z0, const double* A1, double* Z1,
                      const double* A2, double* Z2, int64_t lda, int64_t ldz, double* gpart, hipStream_t st) {
  if (nc <= 0) return 0;
  int64_t blocks = (n + UPD_THREADS - 1) / UPD_THREADS;
#define RIGA_UPD(NQ)                                                                              \
  hipLaunchKernelGGL(k_cgs_update<NQ>, dim3((unsigned)blocks), dim3(UPD_THREADS),                 \
                     (size_t)nc * NQ * sizeof(double), st, n, nc, h,                               \
                     A0, Z0, A1, Z1, A2, Z2, lda, ldz, gpart)
  switch (nq) {
    case 1: RIGA_UPD(1); break;
    case 2: RIGA_UPD(2); break;
    case 3: RIGA_UPD(3); break;
    default: RIGA_UPD(4); break;
  }
#undef RIGA_UPD
  return (int)blocks;
}

// ---------------------------------------------------------------------------
// Pass 1 update fused with the pass 2 products (cgs_tile_update in
// krylov_dev.hpp): each workgroup takes every gridDim.x-th 64-row tile and
// leaves one partial sum per output (c, q) in partial[(c nq + q) nblk + block]
// for k_dots_final.
template <int NQ, int NW, int CPW>
__global__ __launch_bounds__(NW * 64) void k_cgs_upd_dots(int64_t n, int nc, const double* __restrict__ h,
                                                          const double* __restrict__ Vu,
                                                          const double* __restrict__ Vl,
                                                          const double* __restrict__ Wl, int64_t lda,
                                                          double* __restrict__ Zu, double* __restrict__ Zl,
                                                          double* __restrict__ Zw, int64_t ldz,
                                                          double* __restrict__ partial) {
  __shared__ double hs[NW * CPW * NQ];
  __shared__ double red[NW * 3 * NQ * 64];
  __shared__ double fin[3 * NQ * 64];
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
    cgs_tile_update<NQ, NW, CPW>(r0, min(n, r0 + 64), nc, hs, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, red, fin, lane,
                                 wave, acc);
  }
  const int nblk = gridDim.x, blk = blockIdx.x;
  const int c0 = wave * CPW;
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double v = wave_sum(acc[j][q]);
      if (lane == 0 && c0 + j < nc) partial[((int64_t)(c0 + j) * NQ + q) * nblk + blk] = v;
    }
}

bool cgs_tile_fits(int nc, int nq) {
  return nc > 0 && nq >= 1 && nq <= 4 &&
         (nc <= CGS_NARROW_W * CGS_NARROW_C || (nq <= 2 && nc <= CGS_WIDE_W * CGS_WIDE_C));
}

// The wide shape only for up to two block columns (register budget).
template <int NQ>
void launch_cgs_upd_dots(bool narrow, int blocks, int64_t n, int nc, const double* h, const double* Vu,
                         const double* Vl, const double* Wl, int64_t lda, double* Zu, double* Zl, double* Zw,
                         int64_t ldz, double* partial, hipStream_t st) {
  if constexpr (NQ <= 2) {
    if (!narrow) {
      hipLaunchKernelGGL((k_cgs_upd_dots<NQ, CGS_WIDE_W, CGS_WIDE_C>), dim3(blocks), dim3(CGS_WIDE_W * 64), 0, st,
                         n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial);
      return;
    }
  }
  hipLaunchKernelGGL((k_cgs_upd_dots<NQ, CGS_NARROW_W, CGS_NARROW_C>), dim3(blocks), dim3(CGS_NARROW_W * 64), 0,
                     st, n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial);
}

int launch_cgs_update_dots(int64_t n, int nc, int nq, const double* h, const double* Vu, const double* Vl,
                           const double* Wl, int64_t lda, double* Zu, double* Zl, double* Zw, int64_t ldz,
                           double* partial, double* out, hipStream_t st) {
  if (!cgs_tile_fits(nc, nq) || n <= 0) return -1;
  const int64_t ntiles = (n + 63) / 64;
  const int64_t per = (ntiles + CGS_MAX_BLOCKS - 1) / CGS_MAX_BLOCKS;
  const int blocks = (int)((ntiles + per - 1) / per);
  const bool narrow = nc <= CGS_NARROW_W * CGS_NARROW_C;
  switch (nq) {
    case 1: launch_cgs_upd_dots<1>(narrow, blocks, n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial, st); break;
    case 2: launch_cgs_upd_dots<2>(narrow, blocks, n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial, st); break;
    case 3: launch_cgs_upd_dots<3>(narrow, blocks, n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial, st); break;
    default: launch_cgs_upd_dots<4>(narrow, blocks, n, nc, h, Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, partial, st); break;
  }
  const int nout = nc * nq;
  hipLaunchKernelGGL(k_dots_final, dim3((nout + 3) / 4), dim3(256), 0, st, nout, blocks, partial, out);
  return blocks;
}

// ---------------------------------------------------------------------------
// Block Gram--Schmidt with the second pass delayed by one step (block size
// NB <= 2).  At a step the basis holds the finished columns V = V[:, 0:k] and
// the pending block Y = V[:, k:k+NB], the previous image projected once (not
// normalised), and W = S Y is the operator applied to it.  One read of [V Y]
// forms the products of both blocks, one read updates both: Y is finished (its
// second pass and its normalisation) and W is projected once against the
// finished basis, so a step reads the basis twice where two full passes per
// step read it three times, and no separate normalisation pass is needed.
//   k_dcgs_dots    P = [V Y]^T_B [Y W] ((k + NB) x 2NB, output-major;
//                  Vu^T Xu + (M Vl)^T Xl as k_dots) and, on the tensor grid,
//                  M W_l sum-factorised in the same launch (as k_dots_mr);
//   k_dcgs_coef    one workgroup: with s = V^T Y, T^T T = Y^T Y - s^T s, the
//                  finished block V_j = (Y - V s) T^{-1}.  S V_j = (W - S V s)
//                  T^{-1}, where S V = V H00 + Y H10 (the projected matrix's
//                  rows 0..k+NB of columns 0..k); its coefficients on V and V_j
//                  are a = (p - H00 s - s z) T^{-1} and d = T^{-T} (Y^T W -
//                  s^T p) T^{-1} - T z T^{-1} (p = V^T W, z = H10 s), and W' =
//                  S V_j - V a - V_j d = W T^{-1} - V h_v - Y h_y with h_v =
//                  (p - s z) T^{-1} - s T^{-1} d, h_y = z T^{-1} + T^{-1} d.
//                  The earlier columns are rewritten for V_j: H00 += s H10,
//                  H10 <- T H10.  Writes the update coefficients hc, T^{-1},
//                  and H's new column block (a; d; I: W' is the next pending
//                  block as it stands); T not positive beyond rounding (the
//                  block lies in the span of V) sets *flag = 1;
//   k_dcgs_update  per row: W' = W T^{-1} - [V Y] hc_w into V[:, k+NB:k+2NB]
//                  and Y <- -[V Y] hc_y in place (Y's own coefficients
//                  -T^{-1}).
// Without W (the end of a cycle) the same kernels only finish Y.
template <int NB, bool HASW>
__global__ __launch_bounds__(256) void k_dcgs_dots(int64_t n, int nc, const double* __restrict__ Vu,
                                                   const double* __restrict__ Wl, int64_t lda,
                                                   const double* __restrict__ Yu, const double* __restrict__ Yl,
                                                   const double* __restrict__ Ru, const double* __restrict__ Rl,
                                                   double* __restrict__ partial, int nblk, int tn, int p,
                                                   const double* __restrict__ M1, double* __restrict__ MRl) {
  constexpr int NQ = HASW ? 2 * NB : NB;
  extern __shared__ double sm[];
  const int bx = blockIdx.x;
  if (bx < nblk) {
    const int64_t per = (n + nblk - 1) / nblk;
    const int64_t i0 = (int64_t)bx * per;
    const int64_t i1 = min(n, i0 + per);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    dots_body<NQ, 4>(i0, i1, nc, Vu, Wl, lda, Yu, Yl, lda, NB, Ru, Rl, lane, wave,
                     [&](int c, int q, double v) { partial[((int64_t)c * NQ + q) * nblk + bx] = v; });
  } else if (HASW) {
    const int t = bx - nblk, gx = (tn + TT_I - 1) / TT_I;
    tensor_tile<NB, false, TT_J1>(tn, p, (t % gx) * TT_I, (t / gx) * TT_J1, M1, nullptr, 1.0, 0.0, Rl, lda, MRl,
                                  lda, nullptr, 0, 0.0, sm);
  }
}

template <int NB, bool HASW>
__global__ __launch_bounds__(1024) void k_dcgs_coef(int k, const double* __restrict__ P, double* __restrict__ H,
                                                   int ldh, double* __restrict__ hc, double* __restrict__ Xm,
                                                   int* __restrict__ flag) {
  constexpr int NQ = HASW ? 2 * NB : NB;
  constexpr int OFF = HASW ? NB : 0;   // the Y coefficients' first column in hc
  // dynamic shared memory: s (k x NB), H10 (NB x k), u = H00 s (k x NB),
  // p = V^T W (k x NB)
  extern __shared__ double sh[];
  double* ss = sh;
  double* h10 = sh + (size_t)k * NB;
  double* u = h10 + (size_t)k * NB;
  double* pp = u + (size_t)k * NB;
  __shared__ unsigned long long nzmask[4];   // columns c < k where H10 is not zero
  __shared__ double part[4][256][NB];
  __shared__ double z[NB][NB], sts[NB][NB], stp[NB][NB], T[NB][NB], Ti[NB][NB], d[NB][NB], zc[NB][NB];
  __shared__ double py[NB][NQ];   // the rows of P at Y: Y^T Y (and Y^T W)
  __shared__ double hn[NB];       // squared norms of Y's projection coefficients (H's column block k-NB..k)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int t = tid; t < k * NB; t += blockDim.x) {
    const int c = t / NB, e = t % NB;
    ss[t] = P[c * NQ + e];
    if (HASW) pp[t] = P[c * NQ + NB + e];
    h10[e * k + c] = H[k + e + (int64_t)c * ldh];
  }
  if (tid < NB * NQ) py[tid / NQ][tid % NQ] = P[(k + tid / NQ) * NQ + tid % NQ];
  if (wv >= 4 && wv < 4 + NB) {
    // Y = the projected image of the previous block, not normalised: its norm
    // before projection adds these coefficients (read before the rewrite below)
    const int q = wv - 4;
    double a = 0.0;
    if (k >= NB)
      for (int c = lane; c < k; c += 64) {
        const double h = H[c + (int64_t)(k - NB + q) * ldh];
        a += h * h;
      }
    a = wave_sum(a);
    if (lane == 0) hn[q] = a;
  }
  __syncthreads();
  if (tid < 256) {
    bool nz = false;
    if (tid < k)
#pragma unroll
      for (int e = 0; e < NB; ++e) nz = nz || h10[e * k + tid] != 0.0;
    const unsigned long long m = __ballot(nz);
    if (lane == 0) nzmask[wv] = m;
  }
  __syncthreads();
  // u = H00 s and z = H10 s from the projected matrix as it stands: thread
  // (row r, group g) sums a quarter of the columns, eight loads at a time
  {
    const int r = tid & 255, g = tid >> 8;
    const int per = (k + 3) / 4, c0 = g * per, c1 = min(k, c0 + per);
    double acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = 0.0;
    if (r < k + NB) {
#pragma unroll 8
      for (int c = c0; c < c1; ++c) {
        const double hv = H[r + (int64_t)c * ldh];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] += hv * ss[c * NB + q];
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) part[g][r][q] = acc[q];
    __syncthreads();
    if (tid < k + NB) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const double v = part[0][tid][q] + part[1][tid][q] + part[2][tid][q] + part[3][tid][q];
        if (tid < k) u[tid * NB + q] = v;
        else z[tid - k][q] = v;
      }
    }
    __syncthreads();
  }
  // s^T s and s^T p (wave 0; lanes stride the basis columns)
  if (wv == 0) {
    for (int e = 0; e < NB; ++e)
      for (int q = 0; q < NB; ++q) {
        double a = 0.0, b = 0.0;
        for (int c = lane; c < k; c += 64) {
          a += ss[c * NB + e] * ss[c * NB + q];
          if (HASW) b += ss[c * NB + e] * pp[c * NB + q];
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) { sts[e][q] = a; stp[e][q] = b; }
      }
  }
  __syncthreads();
  if (tid == 0) {
    // T^T T = Y^T Y - s^T s (T upper), Ti = T^{-1}; a column keeping at most
    // 1e-12 of its norm before both projections marks a breakdown
    bool bad = false;
    for (int i = 0; i < NB; ++i)
      for (int j = 0; j < NB; ++j) { T[i][j] = 0.0; Ti[i][j] = 0.0; }
    for (int j = 0; j < NB; ++j) {
      const double gjj = py[j][j] + hn[j];
      for (int i = 0; i <= j; ++i) {
        double a = 0.5 * (py[i][j] + py[j][i]) - 0.5 * (sts[i][j] + sts[j][i]);
        for (int kk = 0; kk < i; ++kk) a -= T[kk][i] * T[kk][j];
        if (i == j) {
          if (!(a > 1e-24 * gjj)) { bad = true; a = 1.0; }
          T[j][j] = sqrt(a);
        } else {
          T[i][j] = a / T[i][i];
        }
      }
    }
    for (int j = 0; j < NB; ++j) {
      Ti[j][j] = 1.0 / T[j][j];
      for (int i = j - 1; i >= 0; --i) {
        double a = 0.0;
        for (int kk = i + 1; kk <= j; ++kk) a += T[i][kk] * Ti[kk][j];
        Ti[i][j] = -a / T[i][i];
      }
    }
    if (HASW) {
      // d = Ti^T (Y^T W - s^T p) Ti - T z Ti;  zc = z Ti + Ti d
      double ym[NB][NB], yt[NB][NB], zt[NB][NB];
      for (int e = 0; e < NB; ++e)
        for (int q = 0; q < NB; ++q) ym[e][q] = py[e][(NQ - NB) + q] - stp[e][q];
      for (int e = 0; e < NB; ++e)
        for (int q = 0; q < NB; ++q) {
          double a = 0.0, b = 0.0;
          for (int f = 0; f < NB; ++f) { a += ym[e][f] * Ti[f][q]; b += z[e][f] * Ti[f][q]; }
          yt[e][q] = a;
          zt[e][q] = b;
        }
      for (int e = 0; e < NB; ++e)
        for (int q = 0; q < NB; ++q) {
          double a = 0.0;
          for (int f = 0; f < NB; ++f) a += Ti[f][e] * yt[f][q] - T[e][f] * zt[f][q];
          d[e][q] = a;
        }
      for (int e = 0; e < NB; ++e)
        for (int q = 0; q < NB; ++q) {
          double a = zt[e][q];
          for (int f = 0; f < NB; ++f) a += Ti[e][f] * d[f][q];
          zc[e][q] = a;
          Xm[e * NB + q] = Ti[e][q];
        }
    }
    if (bad) *flag = 1;
  }
  __syncthreads();
  // coefficients, one basis row c per thread
  for (int c = tid; c < k + NB; c += blockDim.x) {
    if (c < k) {
      double sv[NB], sti[NB];
#pragma unroll
      for (int e = 0; e < NB; ++e) sv[e] = ss[c * NB + e];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < NB; ++e) a += sv[e] * Ti[e][q];
        sti[q] = a;
        hc[c * NQ + OFF + q] = a;
      }
      if (HASW) {
        double psz[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
          double a = pp[c * NB + e];
#pragma unroll
          for (int f = 0; f < NB; ++f) a -= sv[f] * z[f][e];
          psz[e] = a;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          double hv = 0.0, av = 0.0;
#pragma unroll
          for (int e = 0; e < NB; ++e) {
            hv += psz[e] * Ti[e][q] - sti[e] * d[e][q];
            av += (psz[e] - u[c * NB + e]) * Ti[e][q];
          }
          hc[c * NQ + q] = hv;
          H[c + (int64_t)(k + q) * ldh] = av;
        }
      }
    } else {
      const int e = c - k;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        hc[c * NQ + OFF + q] = -Ti[e][q];
        if (HASW) {
          hc[c * NQ + q] = zc[e][q];
          H[c + (int64_t)(k + q) * ldh] = d[e][q];
          // the next pending block is W' itself: coefficient I
          H[k + NB + e + (int64_t)(k + q) * ldh] = e == q ? 1.0 : 0.0;
        }
      }
    }
  }
  // the earlier columns in terms of V_j: H00 += s H10 over the columns where
  // H10 is not zero (the last block column after a plain step, all of them
  // after a restart), one row per thread; then H10 <- T H10
  for (int w = 0; w < 4; ++w) {
    unsigned long long m = nzmask[w];
    while (m != 0ull) {
      const int c = w * 64 + __ffsll((long long)m) - 1;
      m &= m - 1ull;
      for (int r = tid; r < k; r += blockDim.x) {
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < NB; ++e) a += ss[r * NB + e] * h10[e * k + c];
        H[r + (int64_t)c * ldh] += a;
      }
    }
  }
  for (int c = tid; c < k; c += blockDim.x) {
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      double a = 0.0;
#pragma unroll
      for (int f = 0; f < NB; ++f) a += T[e][f] * h10[f * k + c];
      H[k + e + (int64_t)c * ldh] = a;
    }
  }
}

template <int NB, bool HASW>
__global__ __launch_bounds__(UPD_THREADS) void k_dcgs_update(int64_t n, int k, const double* __restrict__ hc,
                                                             const double* __restrict__ Xm, double* __restrict__ Vu,
                                                             double* __restrict__ Vl, double* __restrict__ Wl,
                                                             int64_t lda, const double* __restrict__ Zu,
                                                             const double* __restrict__ Zl,
                                                             const double* __restrict__ Zw, int64_t ldz,
                                                             double* __restrict__ Ou, double* __restrict__ Ol,
                                                             double* __restrict__ Ow) {
  constexpr int NQ = HASW ? 2 * NB : NB;
  constexpr int OFF = HASW ? NB : 0;
  extern __shared__ double hs[];
  __shared__ double xm[NB * NB];
  const int nc = k + NB;
  for (int t = threadIdx.x; t < nc * NQ; t += UPD_THREADS) hs[t] = hc[t];
  if (HASW && threadIdx.x < NB * NB) xm[threadIdx.x] = Xm[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x;
  double w0[NB], w1[NB], w2[NB];
  if (i < n) {
    double y0[NB], y1[NB], y2[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) { y0[q] = 0.0; y1[q] = 0.0; y2[q] = 0.0; w0[q] = 0.0; w1[q] = 0.0; w2[q] = 0.0; }
    if (HASW) {
      double r0[NB], r1[NB], r2[NB];
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        r0[e] = Zu[i + e * ldz];
        r1[e] = Zl[i + e * ldz];
        r2[e] = Zw[i + e * ldz];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int e = 0; e < NB; ++e) {
          const double x = xm[e * NB + q];
          w0[q] += r0[e] * x;
          w1[q] += r1[e] * x;
          w2[q] += r2[e] * x;
        }
    }
    for (int c0 = 0; c0 < nc; c0 += UPD_U) {
      double a0[UPD_U], a1[UPD_U], a2[UPD_U];
#pragma unroll
      for (int e = 0; e < UPD_U; ++e) {
        const bool in = c0 + e < nc;
        const int64_t o = i + (int64_t)(c0 + e) * lda;
        a0[e] = in ? Vu[o] : 0.0;
        a1[e] = in ? Vl[o] : 0.0;
        a2[e] = in ? Wl[o] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < UPD_U; ++e) {
        if (c0 + e >= nc) break;
        const double* hr = hs + (c0 + e) * NQ;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (HASW) {
            w0[q] -= a0[e] * hr[q];
            w1[q] -= a1[e] * hr[q];
            w2[q] -= a2[e] * hr[q];
          }
          y0[q] -= a0[e] * hr[OFF + q];
          y1[q] -= a1[e] * hr[OFF + q];
          y2[q] -= a2[e] * hr[OFF + q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int64_t o = i + (int64_t)(k + q) * lda;
      Vu[o] = y0[q];
      Vl[o] = y1[q];
      Wl[o] = y2[q];
      if (HASW) {
        Ou[i + q * lda] = w0[q];
        Ol[i + q * lda] = w1[q];
        Ow[i + q * lda] = w2[q];
      }
    }
  }
}

void launch_dcgs_dots(int64_t n, int k, int nb, bool hasw, const double* Vu, const double* Vl, const double* Wl,
                      int64_t lda, const double* Ru, const double* Rl, double* partial, double* out,
                      const DevSpace* s, const double* M1, double* MRl, hipStream_t st) {
  const int blocks = dots_blocks(n);
  const int nc = k + nb;
  const int tn = (hasw && s != nullptr) ? s->n : 0;
  const int gx = (tn + TT_I - 1) / TT_I, gy = (tn + TT_J1 - 1) / TT_J1;
  const unsigned grid = (unsigned)(blocks + (tn > 0 ? gx * gy : 0));
  const size_t shm = tn > 0 ? tensor_shm(s->p, nb, false, TT_J1) : 0;
  const int p = s != nullptr ? s->p : 0;
  const double* Yu = Vu + (int64_t)k * lda;
  const double* Yl = Vl + (int64_t)k * lda;
#define RIGA_DCD(NB, W)                                                                                         \
  hipLaunchKernelGGL((k_dcgs_dots<NB, W>), dim3(grid), dim3(256), shm, st, n, nc, Vu, Wl, lda, Yu, Yl, Ru, Rl, \
                     partial, blocks, tn, p, M1, MRl)
  if (nb == 1) {
    if (hasw) RIGA_DCD(1, true); else RIGA_DCD(1, false);
  } else {
    if (hasw) RIGA_DCD(2, true); else RIGA_DCD(2, false);
  }
#undef RIGA_DCD
  const int nout = nc * (hasw ? 2 * nb : nb);
  hipLaunchKernelGGL(k_dots_final, dim3((nout + 3) / 4), dim3(256), 0, st, nout, blocks, partial, out);
}

void launch_dcgs_coef(int k, int nb, bool hasw, const double* P, double* H, int ldh, double* hc, double* Xm,
                      int* flag, hipStream_t st) {
  const size_t shm = (size_t)4 * std::max(k, 1) * nb * sizeof(double);
#define RIGA_DCC(NB, W) \
  hipLaunchKernelGGL((k_dcgs_coef<NB, W>), dim3(1), dim3(1024), shm, st, k, P, H, ldh, hc, Xm, flag)
  if (nb == 1) {
    if (hasw) RIGA_DCC(1, true); else RIGA_DCC(1, false);
  } else {
    if (hasw) RIGA_DCC(2, true); else RIGA_DCC(2, false);
  }
#undef RIGA_DCC
}

void launch_dcgs_update(int64_t n, int k, int nb, bool hasw, const double* hc, const double* Xm, double* Vu,
                        double* Vl, double* Wl, int64_t lda, const double* Zu, const double* Zl, const double* Zw,
                        int64_t ldz, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, (n + UPD_THREADS - 1) / UPD_THREADS);
  const size_t shm = (size_t)(k + nb) * (hasw ? 2 * nb : nb) * sizeof(double);
#define RIGA_DCU(NB, W)                                                                                        \
  hipLaunchKernelGGL((k_dcgs_update<NB, W>), dim3((unsigned)blocks), dim3(UPD_THREADS), shm, st, n, k, hc, Xm, \
                     Vu, Vl, Wl, lda, Zu, Zl, Zw, ldz, Vu + (int64_t)(k + nb) * lda,                    \
                     Vl + (int64_t)(k + nb) * lda, Wl + (int64_t)(k + nb) * lda)
  if (nb == 1) {
    if (hasw) RIGA_DCU(1, true); else RIGA_DCU(1, false);
  } else {
    if (hasw) RIGA_DCU(2, true); else RIGA_DCU(2, false);
  }
#undef RIGA_DCU
}

// ---------------------------------------------------------------------------
// Out = In * Q for a tall In (n x kin) and a small Q (kin x kout), one 64-row
// tile per workgroup (body in krylov_dev.hpp).
constexpr int GEMM_WAVES = 8;   // 128 rows per block, one 16-row slab per wave

__global__ __launch_bounds__(GEMM_WAVES * 64) void k_gemm_tall(
    int64_t n, const double* __restrict__ In, int64_t ldi, int kin, const double* __restrict__ Q,
    int kout, double* __restrict__ Out, int64_t ldo) {
  extern __shared__ double qs[];
  const int64_t r0 = (int64_t)blockIdx.x * (16 * GEMM_WAVES);
  gemm_rows_mfma<GEMM_WAVES, 1>(r0, min(n, r0 + 16 * GEMM_WAVES), In, ldi, kin, Q, kout, Out, ldo, qs);
}

void launch_gemm_tall(int64_t n, const double* In, int64_t ldi, int kin, const double* Q, int kout,
                      double* Out, int64_t ldo, hipStream_t st) {
  if (kout <= 0 || kin <= 0 || n <= 0) return;
  const int64_t blocks = (n + 16 * GEMM_WAVES - 1) / (16 * GEMM_WAVES);
  // 64 columns of Q in LDS: at most 64 x 257 doubles (kin <= 254), within the 160 KiB of a CU
  const size_t shm = (size_t)gemm_lds_doubles(kin) * sizeof(double);
  hipLaunchKernelGGL(k_gemm_tall, dim3((unsigned)blocks), dim3(GEMM_WAVES * 64), shm, st, n, In, ldi, kin, Q,
                     kout, Out, ldo);
}

// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_random_fill(double* X, int64_t n, int ncols, int64_t ld, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < ncols; ++c) {
    uint64_t z = splitmix64(seed * 0x100000001B3ull + (uint64_t)c * (uint64_t)n + (uint64_t)i);
    // 53 random bits -> uniform in (-1, 1)
    X[i + c * ld] = 2.0 * (((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

void launch_random_fill(double* X, int64_t n, int ncols, int64_t ld, uint64_t seed, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_random_fill, dim3((unsigned)blocks), dim3(256), 0, st, X, n, ncols, ld, seed);
}

// ---------------------------------------------------------------------------
// Per-pair reductions for the returned eigenvectors u_k = a_k + i b_k, stored
// planar: P[:, k] = a_k, P[:, nv + k] = b_k, and likewise for M P, C P, K P.
// Block (x, k) sums rows of its slice into part[(k * nsplit + x) * 11 + f]:
//   f: aMa bMb aMb aCa bCb aCb aKa bKb aKb aa bb
__global__ __launch_bounds__(256) void k_pair_forms(int64_t n, int nv, const double* __restrict__ P,
                                                    const double* __restrict__ MP, const double* __restrict__ CP,
                                                    const double* __restrict__ KP, int64_t ld,
                                                    double* __restrict__ part) {
  const int k = blockIdx.y, nsplit = gridDim.x;
  const int64_t per = (n + nsplit - 1) / nsplit;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  double f[11];
#pragma unroll
  for (int t = 0; t < 11; ++t) f[t] = 0.0;
  const int64_t ca = (int64_t)k * ld, cb = (int64_t)(nv + k) * ld;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double a = P[ca + i], b = P[cb + i];
    const double ma = MP[ca + i], mb = MP[cb + i];
    const double cA = CP[ca + i], cB = CP[cb + i];
    const double ka = KP[ca + i], kb = KP[cb + i];
    f[0] += a * ma; f[1] += b * mb; f[2] += a * mb;
    f[3] += a * cA; f[4] += b * cB; f[5] += a * cB;
    f[6] += a * ka; f[7] += b * kb; f[8] += a * kb;
    f[9] += a * a;  f[10] += b * b;
  }
  __shared__ double red[11][256];
#pragma unroll
  for (int t = 0; t < 11; ++t) red[t][threadIdx.x] = f[t];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int t = 0; t < 11; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 11) part[((int64_t)k * nsplit + blockIdx.x) * 11 + threadIdx.x] = red[threadIdx.x][0];
}

void launch_pair_forms(int64_t n, int nv, const double* P, const double* MP, const double* CP,
                       const double* KP, int64_t ld, double* part, int nsplit, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_forms, dim3(nsplit, nv), dim3(256), 0, st, n, nv, P, MP, CP, KP, ld, part);
}

// b_k^T (C a_k) per pair (a_k = P column k, b_k = column nv + k, CP = C P):
// part[k * nsplit + x] for split x, summed in a fixed order.
__global__ __launch_bounds__(256) void k_cross_form(int64_t n, int nv, const double* __restrict__ P,
                                                    const double* __restrict__ CP, int64_t ld,
                                                    double* __restrict__ part) {
  const int k = blockIdx.y, nsplit = gridDim.x;
  const int64_t per = (n + nsplit - 1) / nsplit;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  const int64_t ca = (int64_t)k * ld, cb = (int64_t)(nv + k) * ld;
  double f = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) f += P[cb + i] * CP[ca + i];
  __shared__ double red[256];
  red[threadIdx.x] = f;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)k * nsplit + blockIdx.x] = red[0];
}

void launch_cross_form(int64_t n, int nv, const double* P, const double* CP, int64_t ld, double* part, int nsplit,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_cross_form, dim3(nsplit, nv), dim3(256), 0, st, n, nv, P, CP, ld, part);
}

// ||K u + lam C u + lam^2 M u||^2 per pair (lam[2k], lam[2k+1] = re, im) and
// max |u_i|^2 with its index and value:
// part[(k * nsplit + x) * 5 + {0: sum, 1: max, 2: index, 3: re u_i, 4: im u_i}]
__global__ __launch_bounds__(256) void k_pair_resid(int64_t n, int nv, const double* __restrict__ P,
                                                    const double* __restrict__ MP, const double* __restrict__ CP,
                                                    const double* __restrict__ KP, int64_t ld,
                                                    const double* __restrict__ lam, double* __restrict__ part) {
  const int k = blockIdx.y, nsplit = gridDim.x;
  const int64_t per = (n + nsplit - 1) / nsplit;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  const double lr = lam[2 * k], li = lam[2 * k + 1];
  const double l2r = lr * lr - li * li, l2i = 2.0 * lr * li;
  const int64_t ca = (int64_t)k * ld, cb = (int64_t)(nv + k) * ld;
  double s = 0.0, best = -1.0;
  int64_t bi = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double ka = KP[ca + i], kb = KP[cb + i];
    const double cA = CP[ca + i], cB = CP[cb + i];
    const double ma = MP[ca + i], mb = MP[cb + i];
    const double rr = ka + (lr * cA - li * cB) + (l2r * ma - l2i * mb);
    const double ri = kb + (lr * cB + li * cA) + (l2r * mb + l2i * ma);
    s += rr * rr + ri * ri;
    const double a = P[ca + i], b = P[cb + i];
    const double m = a * a + b * b;
    if (m > best) { best = m; bi = i; }
  }
  __shared__ double rs[256], rv[256];
  __shared__ int64_t ri_[256];
  rs[threadIdx.x] = s; rv[threadIdx.x] = best; ri_[threadIdx.x] = bi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      rs[threadIdx.x] += rs[threadIdx.x + st];
      double o = rv[threadIdx.x + st];
      int64_t oi = ri_[threadIdx.x + st];
      if (o > rv[threadIdx.x] || (o == rv[threadIdx.x] && oi < ri_[threadIdx.x])) {
        rv[threadIdx.x] = o; ri_[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)k * nsplit + blockIdx.x) * 5;
    o[0] = rs[0]; o[1] = rv[0]; o[2] = (double)ri_[0];
    o[3] = P[ca + ri_[0]]; o[4] = P[cb + ri_[0]];
  }
}

void launch_pair_resid(int64_t n, int nv, const double* P, const double* MP, const double* CP,
                       const double* KP, int64_t ld, const double* lam, double* part, int nsplit,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pair_resid, dim3(nsplit, nv), dim3(256), 0, st, n, nv, P, MP, CP, KP, ld, lam, part);
}

// X[2 (i + k n) + {0,1}] = s_k (a_j + i b_j) with j = src[k] (s[3k], s[3k+1] the
// complex scale, s[3k+2] the source column): scaled eigenvectors in output
// order, interleaved complex; P has nv planar pairs.
__global__ void k_finalize(int64_t n, int nv, int nout, const double* __restrict__ P, int64_t ld,
                           const double* __restrict__ s, double* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < nout; ++k) {
    const int j = (int)s[3 * k + 2];
    const double a = P[(int64_t)j * ld + i], b = P[(int64_t)(nv + j) * ld + i];
    const double sr = s[3 * k], si = s[3 * k + 1];
    X[2 * ((int64_t)k * n + i)] = a * sr - b * si;
    X[2 * ((int64_t)k * n + i) + 1] = a * si + b * sr;
  }
}

void launch_finalize(int64_t n, int nv, int nout, const double* P, int64_t ld, const double* s, double* X,
                     hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(256), 0, st, n, nv, nout, P, ld, s, X);
}

// Largest absolute row sums of three CSR value arrays sharing one row-pointer
// array (the 1-norms of symmetric matrices), per block of rows: block b covers
// rows rb[b].y .. rb[b].z (or rows b * rows_per_block .. when rb is null) and
// writes part[3 b + a] for array a.  16 lanes per row, every row's loads of
// the three arrays in flight together.
__global__ __launch_bounds__(256) void k_rowabs3(const int4* __restrict__ rb, int64_t ndof, int rows_per_block,
                                                 const int64_t* __restrict__ rowptr, const double* __restrict__ A0,
                                                 const double* __restrict__ A1, const double* __restrict__ A2,
                                                 double* __restrict__ part) {
  int64_t r0, r1;
  if (rb != nullptr) {
    const int4 b = rb[blockIdx.x];
    r0 = b.y; r1 = b.z;
  } else {
    r0 = (int64_t)blockIdx.x * rows_per_block;
    r1 = min(ndof, r0 + rows_per_block);
  }
  const int g = threadIdx.x % 16;
  double best[3] = {0.0, 0.0, 0.0};
  for (int64_t r = r0 + threadIdx.x / 16; r < r1; r += 16) {
    const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t k = k0 + g; k < k1; k += 16) {
      s[0] += fabs(A0[k]);
      s[1] += fabs(A1[k]);
      s[2] += fabs(A2[k]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) s[a] += __shfl_xor(s[a], off, 16);
      best[a] = fmax(best[a], s[a]);
    }
  }
  __shared__ double red[3][256];
#pragma unroll
  for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = best[a];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = fmax(red[a][threadIdx.x], red[a][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 3) part[(int64_t)blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

void launch_rowabs3(const int4* rb, int nblocks, int64_t ndof, int rows_per_block, const int64_t* rowptr,
                    const double* A0, const double* A1, const double* A2, double* part, hipStream_t st) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_rowabs3, dim3(nblocks), dim3(256), 0, st, rb, ndof, rows_per_block, rowptr, A0, A1, A2,
                     part);
}

// Out = am M + ac C + ak K on the common CSR pattern: Q(sigma) for the FP64
// residuals of the refined mixed-precision solves, sigma M + C for the operator.
__global__ __launch_bounds__(256) void k_combine3(int64_t nnz, double am, const double* __restrict__ M, double ac,
                                                  const double* __restrict__ C, double ak,
                                                  const double* __restrict__ K, double* __restrict__ Out) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256)
    Out[k] = am * M[k] + ac * C[k] + ak * K[k];
}

void launch_combine3(int64_t nnz, double am, const double* M, double ac, const double* C, double ak,
                     const double* K, double* Out, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((nnz + 255) / 256, 8192);
  hipLaunchKernelGGL(k_combine3, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, nnz, am, M, ac, C,
                     ak, K, Out);
}

// ---------------------------------------------------------------------------
// Device-side end of a block Gram--Schmidt step, fused with the new basis
// block: with h1, h2 (nc x nq, the two projection passes, output-major
// c*nq+q) and G (nq x nq, the B-Gram matrix of the projected block), factor
// G = R^T R and form Out_m = In_m R^{-1} for three (In, Out) pairs.  Every
// workgroup forms R and R^{-1} itself (the same arithmetic in the same order,
// so all agree) from the few values involved; workgroup 0 also writes
// H[0:nc, k+q] = h1 + h2 and H[nc+c, k+q] = R[c][q].  A column whose squared
// B-norm after projection falls below 1e-24 of its norm before projection (an
// invariant subspace was reached) sets *flag = 1; the caller then redoes the
// solve on the host-checked path.  With gpart, G is first summed from gblk
// per-block partials (nq x nq each, block order).
// With many workgroups (gblk large) the per-workgroup sums of the partials
// would cost more than they save: then one workgroup forms R^{-1} into rbuf
// (mode 1, no rows) and the product reads it from there (mode 2).
template <int NQ>
__global__ __launch_bounds__(256) void k_normalize_gemm3(
    int64_t n, int nc, const double* __restrict__ h1, const double* __restrict__ h2,
    const double* __restrict__ G, const double* __restrict__ gpart, int gblk, double* __restrict__ H, int ldh,
    int k, int* __restrict__ flag, double* __restrict__ rbuf, int mode, const double* __restrict__ I0,
    double* __restrict__ O0, const double* __restrict__ I1, double* __restrict__ O1,
    const double* __restrict__ I2, double* __restrict__ O2, int64_t ld) {
  __shared__ double hn[4];
  __shared__ double gs[16];
  __shared__ double X[NQ * NQ];
  if (mode == 2) {
    if (threadIdx.x < NQ * NQ) X[threadIdx.x] = rbuf[threadIdx.x];
    __syncthreads();
  } else {
  if (gpart != nullptr) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int idx = wv; idx < NQ * NQ; idx += blockDim.x / 64) {
      double s = 0.0;
      for (int b = lane; b < gblk; b += 64) s += gpart[(int64_t)b * NQ * NQ + idx];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) gs[idx] = s;
    }
    __syncthreads();
    G = gs;
  }
  const bool first = blockIdx.x == 0;
  block_normalize_body(nc, NQ, h1, h2, G, first ? H : nullptr, ldh, k, X, first ? flag : nullptr, hn);
  __syncthreads();
  if (mode == 1) {
    if (threadIdx.x < NQ * NQ) rbuf[threadIdx.x] = X[threadIdx.x];
    return;
  }
  }
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double q[NQ][NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a)
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[a][c] = X[a + c * NQ];
  const double* Is[3] = {I0, I1, I2};
  double* Os[3] = {O0, O1, O2};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    if (Is[m] == nullptr) continue;   // fewer than three pairs (uniform branch)
    double x[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a) x[a] = Is[m][i + a * ld];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < NQ; ++a) acc += x[a] * q[a][c];
      Os[m][i + c * ld] = acc;
    }
  }
}

void launch_normalize_gemm3(int64_t n, int nc, int nq, const double* h1, const double* h2, const double* G,
                            const double* gpart, int gblk, double* H, int ldh, int k, int* flag, double* rbuf,
                            const double* I0, double* O0, const double* I1, double* O1, const double* I2,
                            double* O2, int64_t ld, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, (n + 255) / 256);
  // fused while every workgroup's share of the partial sums stays small
  const bool split = gpart != nullptr && gblk > 512;
#define RIGA_NG3(NQ, GRID, NROWS, MODE)                                                                      \
  hipLaunchKernelGGL(k_normalize_gemm3<NQ>, dim3((unsigned)(GRID)), dim3(256), 0, st, (int64_t)(NROWS), nc, h1, \
                     h2, G, gpart, gblk, H, ldh, k, flag, rbuf, MODE, I0, O0, I1, O1, I2, O2, ld)
#define RIGA_NG3_ALL(NQ)                                   \
  if (split) {                                             \
    RIGA_NG3(NQ, 1, 0, 1);                                 \
    RIGA_NG3(NQ, blocks, n, 2);                            \
  } else {                                                 \
    RIGA_NG3(NQ, blocks, n, 0);                            \
  }
  switch (nq) {
    case 1: RIGA_NG3_ALL(1); break;
    case 2: RIGA_NG3_ALL(2); break;
    case 3: RIGA_NG3_ALL(3); break;
    default: RIGA_NG3_ALL(4); break;
  }
#undef RIGA_NG3_ALL
#undef RIGA_NG3
}

// ---------------------------------------------------------------------------
// Interleaved complex columns X (n x nv) -> planar P = [Re X | Im X].
__global__ void k_deinterleave(int64_t n, int nv, const double* __restrict__ X, double* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < nv; ++k) {
    P[(int64_t)k * n + i] = X[2 * ((int64_t)k * n + i)];
    P[(int64_t)(nv + k) * n + i] = X[2 * ((int64_t)k * n + i) + 1];
  }
}

void launch_deinterleave(int64_t n, int nv, const double* X, double* P, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_deinterleave, dim3((unsigned)blocks), dim3(256), 0, st, n, nv, X, P);
}

// Element sensitivities of the eigenvalues to a per-element damping field
// C = C0 + sum_e c_e M_e.  For a complex-symmetric pencil the left eigenvector
// is conj(u), so d lam / d c_e = -lam u^T M_e u / u^T (2 lam M + C) u
// (unconjugated transposes).  With w_k = conj(dL/dlam_k) (-lam_k / d_k) given,
// grad[e] = sum_k Re(w_k q_ke), q_ke = u_k^T M_e u_k; M_e = m_ey (x) m_ex from the
// 1-D element tables.  One thread per element; u read from the planar P.
constexpr int MAXP1 = 9;

__global__ __launch_bounds__(256) void k_adjoint(int p, int ne, int n, const int* __restrict__ first,
                                                 const double* __restrict__ tabM, int nv,
                                                 const double* __restrict__ P, int64_t ndof,
                                                 const double* __restrict__ w, double* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ne * ne) return;
  const int ex = (int)(e % ne), ey = (int)(e / ne);
  const int np = p + 1;
  const double* mx = tabM + (int64_t)ex * np * np;
  const double* my = tabM + (int64_t)ey * np * np;
  // Dirichlet index of the local functions (-1: removed boundary function)
  int gx[MAXP1], gy[MAXP1];
  for (int l = 0; l < np; ++l) {
    const int fx = first[ex] + l - 1, fy = first[ey] + l - 1;
    gx[l] = (fx >= 0 && fx < n) ? fx : -1;
    gy[l] = (fy >= 0 && fy < n) ? fy : -1;
  }
  double acc = 0.0;
  for (int k = 0; k < nv; ++k) {
    const double* a = P + (int64_t)k * ndof;
    const double* bi = P + (int64_t)(nv + k) * ndof;
    double ur[MAXP1 * MAXP1], ui[MAXP1 * MAXP1];
    for (int ly = 0; ly < np; ++ly)
      for (int lx = 0; lx < np; ++lx) {
        const bool ok = gx[lx] >= 0 && gy[ly] >= 0;
        const int64_t d = ok ? (int64_t)gy[ly] * n + gx[lx] : 0;
        ur[ly * np + lx] = ok ? a[d] : 0.0;
        ui[ly * np + lx] = ok ? bi[d] : 0.0;
      }
    // t = (m_ey (x) m_ex) u, then q = u^T t (complex, unconjugated)
    double qr = 0.0, qi = 0.0;
    for (int ly = 0; ly < np; ++ly)
      for (int lx = 0; lx < np; ++lx) {
        double tr = 0.0, ti = 0.0;
        for (int my2 = 0; my2 < np; ++my2) {
          double sr = 0.0, si = 0.0;
          for (int mx2 = 0; mx2 < np; ++mx2) {
            const double m = mx[lx * np + mx2];
            sr += m * ur[my2 * np + mx2];
            si += m * ui[my2 * np + mx2];
          }
          const double m = my[ly * np + my2];
          tr += m * sr;
          ti += m * si;
        }
        const double vr = ur[ly * np + lx], vi = ui[ly * np + lx];
        qr += vr * tr - vi * ti;
        qi += vr * ti + vi * tr;
      }
    acc += w[2 * k] * qr - w[2 * k + 1] * qi;   // Re(w q)
  }
  grad[e] = acc;
}

void launch_adjoint(const DevSpace& s, const double* tabM, int nv, const double* P, int64_t ndof,
                    const double* w, double* grad, hipStream_t st) {
  const int64_t ne2 = (int64_t)s.ne * s.ne;
  const int64_t blocks = (ne2 + 255) / 256;
  hipLaunchKernelGGL(k_adjoint, dim3((unsigned)blocks), dim3(256), 0, st, s.p, s.ne, s.n, s.first, tabM, nv, P,
                     ndof, w, grad);
}

}  // namespace riga
