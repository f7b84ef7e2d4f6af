// Multifrontal Cholesky of Q(sigma) = sigma^2 M + sigma C + K over the
// nested-dissection tree (Sec. 3.3: rIGA hyperplanes are the separators;
// Sec. 5.2.1: one factorization per shift).
//
// A front of node v holds its own dofs (eliminated here) followed by its
// boundary dofs (ancestors coupled to the subtree).  Storage per node, at the
// same offset in two buffers of nf x no entries (the front buffer and the
// factor buffer) plus the update block:
//   front   nf x no, column-major (ld nf): the own columns of the assembled
//           front, updated in place by the panels; after the factorization it
//           receives F (row r of F at r * no), the matrix the sweeps use;
//   factor  nf x no, column-major: L (the own columns of the Cholesky factor),
//           written panel by panel (kept apart from the front so that a
//           panel's rows are read by every workgroup of its update launch
//           while the factor rows are written);
//   U       nb x nb, column-major: the update (Schur complement) matrix that
//           the parent adds into its front ("extend-add").
// A tree level is processed by a pipeline of batched kernels whose grids span
// every node of the level:
//   k_front_assemble   zero the front and add the original entries of Q
//                      (64 front columns per workgroup);
//   k_front_extend     add the children's update blocks, one child slot per
//                      launch (64 child columns per workgroup);
//   per 64-wide panel of own columns:
//     k_potrf_diag     Cholesky of the 64x64 diagonal block and its inverse
//                      D_k = L_kk^{-1}, both blocked by 16 over four waves
//                      (one workgroup per node, in LDS);
//     k_panel_update   per pair of 64-row tiles (I, J), J <= I, below the
//                      block: the panel rows X_I = A_I D_k^T and X_J (MFMA),
//                      X_I stored as factor rows by the diagonal pair, and
//                      the trailing tile C_IJ -= X_I X_J^T (MFMA);
//     or, on levels with many tile pairs, k_panel_rows (X_I once per row
//                      tile, stored as factor rows) and k_panel_trail (the
//                      tile pairs from the stored rows);
//   k_rtrsm            rows of F = [L_oo^{-1}; L_bo L_oo^{-1}] from
//                      X L_oo = [I; L_bo], block column by block column from
//                      the right with the stored D_k (MFMA, 16 waves);
//   k_pack             F in the two sweep layouts Lp / Tp (16-byte groups of
//                      columns / rows).
// With F, each forward/backward sweep is one matrix-vector product per node.
// Every kernel is a template over the element type E of the node's front:
// double (v_mfma_f64_16x16x4_f64) or float (v_mfma_f32_16x16x4_f32, FP32
// products and accumulation) for the mixed-precision factorization, where the
// lower tree levels are FP32 and the top levels FP64.  Products run on 64x64
// tiles staged in LDS; a tile is split over the waves of the workgroup (4
// waves: 32x32 quadrants of 2x2 MFMA tiles; 16 waves: one 16x16 MFMA tile
// each).
#include "kernels.hpp"
#include "mfma_layout.hpp"

#include <algorithm>

namespace riga {

constexpr int FT = 256;     // threads per workgroup (four waves)
constexpr int TB = 64;      // panel / tile width
constexpr int LDT = TB + 1; // LDS row stride (elements)
// A panel's trailing update forms the panel rows once per row tile
// (k_panel_rows*, then k_panel_trail* over the tile pairs: one product per
// pair) instead of in every tile pair (the fused k_panel_update*: three
// products per pair, one launch) when the level's tile pairs (fronts x pairs)
// number at least SPLIT_MIN_PAIRS, i.e. when the fused kernel would need more
// than one round of workgroups on the chip; below that the second launch
// costs more than the products it saves.
#ifndef SPLIT_MIN_PAIRS
#define SPLIT_MIN_PAIRS 512
#endif

static bool split_panel(int count, int nrc) {
  const long pairs = (long)count * nrc * (nrc + 1) / 2;
  return nrc >= 2 && pairs >= SPLIT_MIN_PAIRS;
}

template <class E>
struct Front {
  E* L; E* U; int nf, no, nb;
  __device__ __forceinline__ E* at(int i, int j) const {  // requires i >= j
    return j < no ? L + (int64_t)j * nf + i : U + (int64_t)(j - no) * nb + (i - no);
  }
};

template <class E>
__device__ __forceinline__ Front<E> front_of(const DevTree& t, int v, E* Lbuf, E* Ubuf) {
  return Front<E>{Lbuf + t.loff[v], Ubuf + t.uoff[v], t.nf[v], t.no[v], t.nb[v]};
}

template <class E> using acc_t = typename Mfma<E>::acc_t;

// A 64 x 64 product tile split over the NW waves of a workgroup: a WR x WC
// grid of wave regions, each TI x TJ MFMA tiles of 16 x 16.
template <class E, int NW>
struct Tile64 {
  static constexpr int WC = NW == 16 ? 4 : 2, WR = NW / WC;
  static constexpr int TI = TB / WR / 16, TJ = TB / WC / 16;
  struct Acc { acc_t<E> a[TI][TJ]; };
  static __device__ __forceinline__ int row(int lane, int wave, int ti, int v) {
    return (wave / WC) * (TB / WR) + 16 * ti + Mfma<E>::drow(lane, v);
  }
  static __device__ __forceinline__ int col(int lane, int wave, int tj) {
    return (wave % WC) * (TB / WC) + 16 * tj + mfma_d_col(lane);
  }
  static __device__ __forceinline__ void zero(Acc& c) {
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) c.a[ti][tj] = acc_t<E>{0, 0, 0, 0};
  }
  // acc += A (64 x kw) B (kw x 64) with both operands read from global memory:
  // A(i, k) at A[k * lda + i] for i < nrows (rows past nrows are zero), B(k, j)
  // at B[k * ldb + j]; k < kw.  Lanes 0..15 of a k row read 16 consecutive
  // entries, and the unrolled k loop keeps several rounds of loads in flight
  // (masked lanes read a valid address and select zero).
  static __device__ __forceinline__ void mma_global(const E* __restrict__ A, int64_t lda, int nrows,
                                                    const E* __restrict__ B, int ldb, int kw, Acc& c, int lane,
                                                    int wave) {
    const int wr = (wave / WC) * (TB / WR), wc = (wave % WC) * (TB / WC);
#pragma unroll 4
    for (int k0 = 0; k0 < TB; k0 += 4) {
      const int k = k0 + mfma_ab_k(lane);
      const bool kin = k < kw;
      E a[TI], b[TJ];
#pragma unroll
      for (int t = 0; t < TI; ++t) {
        const int i = wr + 16 * t + mfma_a_row(lane);
        const bool in = kin && i < nrows;
        const E x = A[in ? (int64_t)k * lda + i : 0];
        a[t] = in ? x : E(0);
      }
#pragma unroll
      for (int t = 0; t < TJ; ++t) {
        const E x = B[kin ? k * ldb + wc + 16 * t + mfma_b_col(lane) : 0];
        b[t] = kin ? x : E(0);
      }
#pragma unroll
      for (int ti = 0; ti < TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) c.a[ti][tj] = Mfma<E>::mma(a[ti], b[tj], c.a[ti][tj]);
    }
  }
  // acc += A (64 x kw) B^T with A and B both stored as row panels in global
  // memory: A(i, k) at A[k * lda + i] for i < nrows, B(j, k) at B[k * ldb + j]
  // for j < ncols (rows past either bound are zero; masked lanes read a valid
  // address and select zero); k < kw.
  static __device__ __forceinline__ void mma_global_nt(const E* __restrict__ A, int64_t lda, int nrows,
                                                       const E* __restrict__ B, int64_t ldb, int ncols, int kw,
                                                       Acc& c, int lane, int wave, const E* kscale = nullptr) {
    const int wr = (wave / WC) * (TB / WR), wc = (wave % WC) * (TB / WC);
#pragma unroll 4
    for (int k0 = 0; k0 < TB; k0 += 4) {
      const int k = k0 + mfma_ab_k(lane);
      const bool kin = k < kw;
      E a[TI], b[TJ];
#pragma unroll
      for (int t = 0; t < TI; ++t) {
        const int i = wr + 16 * t + mfma_a_row(lane);
        const bool in = kin && i < nrows;
        const E x = A[in ? (int64_t)k * lda + i : 0];
        a[t] = in ? x : E(0);
      }
      const E ks = (kscale != nullptr && kin) ? kscale[k] : E(1);
#pragma unroll
      for (int t = 0; t < TJ; ++t) {
        const int j = wc + 16 * t + mfma_b_col(lane);
        const bool in = kin && j < ncols;
        const E x = B[in ? (int64_t)k * ldb + j : 0];
        b[t] = in ? x * ks : E(0);
      }
#pragma unroll
      for (int ti = 0; ti < TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) c.a[ti][tj] = Mfma<E>::mma(a[ti], b[tj], c.a[ti][tj]);
    }
  }
  // acc += sign * A (64 x kw) B (kw x 64), A at As[i * LDT + k], B at Bs[k * LDT + j]
  static __device__ __forceinline__ void mma(const E* As, const E* Bs, int kw, Acc& c, int lane, int wave,
                                             E sign) {
    const int wr = (wave / WC) * (TB / WR), wc = (wave % WC) * (TB / WC);
    for (int k0 = 0; k0 < kw; k0 += 4) {
      const int k = k0 + mfma_ab_k(lane);
      E a[TI], b[TJ];
#pragma unroll
      for (int t = 0; t < TI; ++t) a[t] = (k < kw) ? sign * As[(wr + 16 * t + mfma_a_row(lane)) * LDT + k] : E(0);
#pragma unroll
      for (int t = 0; t < TJ; ++t) b[t] = (k < kw) ? Bs[k * LDT + wc + 16 * t + mfma_b_col(lane)] : E(0);
#pragma unroll
      for (int ti = 0; ti < TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) c.a[ti][tj] = Mfma<E>::mma(a[ti], b[tj], c.a[ti][tj]);
    }
  }
};

// ---------------------------------------------------------------------------------
// Front assembly, columns [64 y, 64 y + 64) of the front per workgroup: zero
// them (own columns in the L block, boundary columns in the U block) and add
// the original entries Q[g, d] for the own dofs d of the chunk and front dofs g
// at or below d (formed in FP64, stored in E).  The node's sorted front keys
// and their positions are staged in shared memory (2 nf ints); each wave takes
// one own column at a time, its lanes the stored entries of that row, and
// finds an entry's front position by binary search in shared memory.
template <class E>
__global__ __launch_bounds__(FT) void k_front_assemble(
    int n, const int* lo, const int* hi, const int64_t* rowptr, const int* __restrict__ col,
    DevTree t, const int* __restrict__ level_nodes, double s2, double s1,
    const double* __restrict__ Kv, const double* __restrict__ Mv, const double* __restrict__ Cv,
    E* __restrict__ Lbuf, E* __restrict__ Ubuf) {
  extern __shared__ int keys[];   // keys[0, nf): sorted front dofs; keys[nf, 2 nf): their positions
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  const int nf = F.nf, no = F.no, nb = F.nb;
  const int c0 = TB * blockIdx.y, c1 = min(nf, c0 + TB);
  if (c0 >= nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int* fd = t.fdofs + t.foff[v];
  const int* fk = t.fkey + t.foff[v];
  const int* fp = t.fpos + t.foff[v];
  int base = 0;   // forest: the node's problem has its own space, shift and dof range
  if (t.inst != nullptr) {
    const int q = t.inst[v];
    const DevSpace& sp = t.spaces[q];
    n = sp.n; lo = sp.lo; hi = sp.hi; rowptr = sp.rowptr;
    base = (int)t.dofbase[q];
    s1 = t.isig[q];
    s2 = s1 * s1;
  }
  const bool own = c0 < no;
  if (own)
    for (int x = tid; x < nf; x += FT) {
      keys[x] = fk[x];
      keys[nf + x] = fp[x];
    }
  for (int c = c0; c < c1; ++c) {
    if (c < no) {
      for (int r = tid; r < nf; r += FT) F.L[(int64_t)c * nf + r] = E(0);
    } else {
      for (int r = tid; r < nb; r += FT) F.U[(int64_t)(c - no) * nb + r] = E(0);
    }
  }
  __syncthreads();
  if (!own) return;
  // the wave's columns a = c0 + wave + 4u (at most 16): lane u fetches the
  // row description of column u first, so the columns' entry loads do not
  // wait on one another's index loads
  const int na = (min(c1, no) - c0 - wave + FT / 64 - 1) / (FT / 64);
  int m_lx = 0, m_wx = 1, m_ly = 0, m_k0 = 0, m_len = 0;
  if (lane < na) {
    const int d = fd[c0 + wave + (FT / 64) * lane] - base;
    if (col == nullptr) {
      const int i = d % n, j = d / n;
      m_lx = lo[i];
      m_wx = hi[i] - m_lx + 1;
      m_ly = lo[j];
    }
    const int64_t r0 = rowptr[d];
    m_k0 = (int)(r0 - rowptr[0]);
    m_len = (int)(rowptr[d + 1] - r0);
  }
  const int64_t kbase = rowptr[0];
  int mlen = m_len;   // longest row of the wave's columns
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mlen = max(mlen, __shfl_xor(mlen, off, 64));
  // chunks of 64 stored entries per row (lane = entry); per batch of eight
  // columns every value load is issued before the first search, so their
  // latencies overlap (lanes past a row's end read the row's first entry)
  constexpr int UB = 8;
  for (int ch = 0; ch * 64 < mlen; ++ch) {
    const int o = ch * 64 + lane;
    for (int u0 = 0; u0 < na; u0 += UB) {
      double q[UB];
#pragma unroll
      for (int uu = 0; uu < UB; ++uu) {
        const int u = min(u0 + uu, 15);
        const int len = u0 + uu < na ? __builtin_amdgcn_readlane(m_len, u) : 0;
        const int64_t k = kbase + __builtin_amdgcn_readlane(m_k0, u) + (o < len ? o : 0);
        q[uu] = s2 * Mv[k] + s1 * Cv[k] + Kv[k];
      }
#pragma unroll
      for (int uu = 0; uu < UB; ++uu) {
        const int u = u0 + uu;
        if (u >= na) break;
        if (o >= __builtin_amdgcn_readlane(m_len, u)) continue;
        const int a = c0 + wave + (FT / 64) * u;
        int g;
        if (col != nullptr) {
          g = col[kbase + __builtin_amdgcn_readlane(m_k0, u) + o] + base;
        } else {
          const int lx = __builtin_amdgcn_readlane(m_lx, u), wx = __builtin_amdgcn_readlane(m_wx, u);
          const int ly = __builtin_amdgcn_readlane(m_ly, u);
          g = (ly + o / wx) * n + lx + o % wx + base;
        }
        int x0 = 0, x1 = nf;  // binary search of g among the sorted front keys
        while (x1 - x0 > 1) {
          const int c = (x0 + x1) >> 1;
          if (keys[c] <= g) x0 = c; else x1 = c;
        }
        if (keys[x0] == g) {
          const int pos = keys[nf + x0];
          if (pos >= a) F.L[(int64_t)a * nf + pos] = (E)q[uu];
        }
      }
    }
  }
}

// Columns [l0, l1) of a child's update block U (nbc x nbc, lower triangle)
// added into the parent front at the mapped positions (mk: the map from child
// row l0 on, in shared memory).  A lane owns rows k and walks the tile's
// columns in batches of sixteen: the front entries are distinct (the map is
// injective), so their loads are all issued before the sums are stored.
template <class E, class S>
__device__ __forceinline__ void extend_tile(const Front<E>& F, const S* __restrict__ Uc, int nbc, int l0, int l1,
                                            const int* mk) {
  constexpr int B = 16;
  for (int k = l0 + (int)threadIdx.x; k < nbc; k += FT) {
    const int pk = mk[k - l0];
    const int lend = min(l1, k + 1);
    for (int l = l0; l < lend; l += B) {
      // columns past lend read the batch's first entry and store nothing
      E* p[B];
      E f[B];
      S u[B];
#pragma unroll
      for (int e = 0; e < B; ++e) {
        const int le = l + e < lend ? l + e : l;
        p[e] = F.at(pk, mk[le - l0]);
        u[e] = Uc[(int64_t)le * nbc + k];
      }
#pragma unroll
      for (int e = 0; e < B; ++e) f[e] = *p[e];
#pragma unroll
      for (int e = 0; e < B; ++e)
        if (l + e < lend) *p[e] = f[e] + (E)u[e];
    }
  }
}

// Extend-add of child number `slot` of every node: child columns [64 y, +64);
// the map from child boundary to parent front positions is injective, so the
// workgroups of one launch write disjoint entries.  A child's update block is
// FP32 (U32) when t.prec marks the child, else FP64 (U64).  Dynamic shared
// memory: the child's map from the tile's first row on (at most max_child_nb
// ints).
template <class E>
__global__ __launch_bounds__(FT) void k_front_extend(DevTree t, const int* __restrict__ level_nodes, int slot,
                                                     E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                     const float* __restrict__ U32,
                                                     const double* __restrict__ U64) {
  extern __shared__ int mk[];
  const int v = level_nodes[blockIdx.x];
  if (t.coff[v] + slot >= t.coff[v + 1]) return;
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  const int c = t.clist[t.coff[v] + slot];
  const int nbc = t.nb[c];
  const int l0 = TB * blockIdx.y, l1 = min(nbc, l0 + TB);
  if (l0 >= nbc) return;
  const int* mp = t.maps + t.moff[c];
  for (int k = l0 + (int)threadIdx.x; k < nbc; k += FT) mk[k - l0] = mp[k];
  __syncthreads();
  if (t.prec != nullptr && t.prec[c])
    extend_tile(F, U32 + t.uoff[c], nbc, l0, l1, mk);
  else
    extend_tile(F, U64 + t.uoff[c], nbc, l0, l1, mk);
}

// ---------------------------------------------------------------------------------
// Entry of register v held by lane l (l uniform), for every lane.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1/sqrt(x) from the hardware estimate refined by Newton steps
// y <- y + y (1 - x y^2) / 2 (two in FP64, one in FP32); x > 0 and normal.
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rsqrt_refined(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float e = fmaf(-x * y, y, 1.0f);
  return fmaf(0.5f * y, e, y);
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky of the diagonal block [k0, k0+w) of the front and D = its inverse
// (lower), stored transposed at D + (doff[v] + k0/64) * 4096 as Dt[c * 64 + r]
// = D[r][c] (zero outside the w x w block), L_kk into the factor buffer.  The block sits in
// LDS, padded to 64 x 64 with the identity.  Both are blocked by 16:
//   factorisation: wave 0 factors a 16-column block column (lane = row: at
//   column c every lane scales its entry, the column is written to LDS, and
//   every lane updates the rest of its row from broadcast reads of it), then
//   all four waves subtract its product from the trailing lower triangle;
//   inverse: wave b inverts diagonal block b by forward substitution (lane =
//   column), then wave j forms the blocks below it in block column j,
//   D_ij = -D_ii sum_k L_ik D_kj, one block row after the other.
// A pivot that is not positive (or NaN) is recorded in *status (the front's
// dof, first one wins) and replaced by 1 so that the kernel completes.
// Signed form (t.sgn not null; an indefinite K - s M, Sec. 4.1.4): the
// factorization is A = L S L^T with S = diag(+-1) the signs of the pivots
// (LDL^T with D = S |D| folded into L, no pivoting): l_cc = sqrt|a_cc|,
// l_rc = a_rc / (s_c l_cc), and the Schur complement keeps a_rj - a_rc a_jc /
// a_cc; the signs go to t.sgn[dof] and their negative count (the inertia of
// Sylvester's law) is added to *negs.  Only a zero or NaN pivot is an error.
template <class E>
__global__ __launch_bounds__(FT) void k_potrf_diag(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                   const E* __restrict__ Lbuf, E* __restrict__ Fbuf,
                                                   E* __restrict__ Dbuf, int64_t* __restrict__ status,
                                                   unsigned long long* __restrict__ negs) {
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v];
  if (no <= k0) return;
  const int w = min(TB, no - k0);
  const E* L = Lbuf + t.loff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E S[TB][LDT];
  __shared__ E Dm[TB][LDT];
  __shared__ E Tx[3][16][17];   // per wave: the product sum_k L_ik D_kj of one block
  __shared__ E rd[TB];          // reciprocal pivots
  __shared__ E sg[TB];          // pivot signs
  const bool sgd = t.sgn != nullptr;
  {
    // every load of the block issued before the first LDS store (coalesced
    // along the column; entries outside the w x w lower triangle read the
    // block's first entry and are replaced)
    constexpr int U = TB * TB / FT;
    E x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = tid + u * FT, r = idx % TB, c = idx / TB;
      const bool in = c <= r && r < w;
      x[u] = L[in ? (int64_t)(k0 + c) * nf + k0 + r : (int64_t)k0 * nf + k0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = tid + u * FT, r = idx % TB, c = idx / TB;
      const bool in = c <= r && r < w;
      S[r][c] = in ? x[u] : ((c == r && r >= w) ? E(1) : E(0));
      Dm[r][c] = E(0);
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < TB; c0 += 16) {
    if (wave == 0) {
      const int r = lane;
      E row[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) row[j] = S[r][c0 + j];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int cc = c0 + c;
        E piv = lane_value(row[c], cc);
        E s = E(1);
        if (sgd && piv < E(0)) {
          s = E(-1);
          piv = -piv;
        }
        if (!(piv > E(0))) {           // not SPD (signed form: zero) or NaN: record, continue with 1
          if (r == cc && cc < w)
            atomicCAS((unsigned long long*)status, (unsigned long long)(-1ll),
                      (unsigned long long)t.fdofs[t.foff[v] + k0 + cc]);
          piv = E(1);
        }
        const E inv = rsqrt_refined(piv);
        const E d = piv * inv;
        if (r == cc) {
          rd[cc] = inv;
          sg[cc] = s;
        }
        const E lrc = row[c] * inv * s;   // L[r][cc] (rows below the pivot)
        row[c] = (r == cc) ? d : lrc;
        // column cc published in LDS; the rest of the block column is
        // updated with a_rj - a_rc a_jc / a_cc = a_rj - s l_rc l_jc, the l_jc
        // read as broadcasts
        if (r >= cc) S[r][cc] = row[c];
        wave_sync();
        const E t = lrc * s;
#pragma unroll
        for (int j = c + 1; j < 16; ++j) row[j] -= t * S[c0 + j][cc];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (r >= c0 + j) S[r][c0 + j] = row[j];
    }
    __syncthreads();
    const int n = TB - c0 - 16;   // trailing rows / columns
    for (int idx = tid; idx < n * n; idx += FT) {
      const int i = idx / n, j = idx % n;
      if (j <= i) {
        const int ri = c0 + 16 + i, rj = c0 + 16 + j;
        E s = S[ri][rj];
#pragma unroll
        for (int c = 0; c < 16; ++c) s -= S[ri][c0 + c] * sg[c0 + c] * S[rj][c0 + c];
        S[ri][rj] = s;
      }
    }
    __syncthreads();
  }
  // inverse: diagonal blocks, wave b takes block b, lane = column (16 lanes)
  if (lane < 16) {
    const int base = 16 * wave, c = lane;
    E dc[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      E sum = E(0);
#pragma unroll
      for (int k = 0; k < rr; ++k) sum += S[base + rr][base + k] * dc[k];
      const E ri = rd[base + rr];
      dc[rr] = (rr < c) ? E(0) : (rr == c ? ri : -sum * ri);
      Dm[base + rr][base + c] = dc[rr];
    }
  }
  __syncthreads();
  // blocks below the diagonal: wave j takes block column j; lane = column c
  // of the block and four consecutive rows 4 rg .. 4 rg + 3
  if (wave < 3) {
    const int j = wave, c = lane & 15, rg = lane >> 4;
    for (int i = j + 1; i < 4; ++i) {
      E tv[4] = {E(0), E(0), E(0), E(0)};
      for (int k = 16 * j; k < 16 * i; ++k) {
        const E dk = Dm[k][16 * j + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) tv[u] += S[16 * i + 4 * rg + u][k] * dk;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) Tx[j][4 * rg + u][c] = tv[u];
      wave_sync();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = 4 * rg + u;
        E s = E(0);
#pragma unroll
        for (int q = 0; q < 16; ++q) s += Dm[16 * i + r][16 * i + q] * Tx[j][q][c];
        Dm[16 * i + r][16 * j + c] = -s;
      }
      wave_sync();
    }
  }
  __syncthreads();
  E* Lf = Fbuf + t.loff[v];
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int r = idx % TB, c = idx / TB;
    if (r < w && c <= r) Lf[(int64_t)(k0 + c) * nf + k0 + r] = S[r][c];
  }
  // D stored transposed: Dt[c * 64 + r] = D[r][c]
  E* Dt = Dbuf + ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int c = idx / TB, r = idx % TB;
    Dt[idx] = (r < w && c < w) ? Dm[r][c] : E(0);
  }
  if (sgd && wave == 0) {
    const bool neg = lane < w && sg[lane] < E(0);
    if (lane < w) t.sgn[t.fdofs[t.foff[v] + k0 + lane]] = (double)sg[lane];
    const unsigned long long cnt = __builtin_popcountll(__ballot(neg));
    if (lane == 0 && cnt > 0) atomicAdd(negs, cnt);
  }
}

// Panel rows and trailing update below the panel [k0, k0 + w), one workgroup
// per pair (I, J), J <= I, of 64-row tiles from s0 = k0 + w (pair index in
// blockIdx.y): X_I = A_I D^T and X_J = A_J D^T from the panel rows A of the
// front (MFMA; the diagonal pair writes X_I into the factor buffer), then
// C_IJ -= X_I X_J^T on the front's lower triangle (MFMA).  Signed form: the
// factor rows are X_I S and the update C_IJ -= X_I S X_J^T (S the panel's
// pivot signs).  No workgroup writes
// what another one reads: the panel is read from the front, X goes to the
// factor buffer, and the C tiles are disjoint.
template <class E>
__global__ __launch_bounds__(FT) void k_panel_update(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                     E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                     E* __restrict__ Fbuf, const E* __restrict__ Dbuf) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  if (F.no <= k0) return;
  const int w = min(TB, F.no - k0);
  const int s0 = k0 + w;
  const int pidx = blockIdx.y;
  int I = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= pidx) ++I;
  while (I * (I + 1) / 2 > pidx) --I;
  const int J = pidx - I * (I + 1) / 2;
  const int rI = s0 + TB * I, rJ = s0 + TB * J;
  if (rI >= F.nf) return;
  const int nf = F.nf;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E Xi[TB * LDT];   // X_I S (A operand; S the panel's pivot signs)
  __shared__ E Xj[TB * LDT];   // X_J^T (B operand)
  __shared__ E ps[TB];
  if (tid < TB) ps[tid] = (t.sgn != nullptr && tid < w) ? (E)t.sgn[t.fdofs[t.foff[v] + k0 + tid]] : E(1);
  // B operand of X = A D^T: D^T(k, j) = Dt[k * 64 + j], row-major in global memory
  const E* Dt = Dbuf + ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  // the C tile's current values, loaded before the products so that their
  // latency overlaps them (entries outside the lower triangle read the tile's
  // corner and are not used)
  typename TL::Acc c;
  E* cp[TL::TI][TL::TJ][4];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rI + TL::row(lane, wave, ti, e), cc = rJ + TL::col(lane, wave, tj);
        const bool in = r < nf && cc < nf && r >= cc;
        cp[ti][tj][e] = in ? F.at(r, cc) : nullptr;
        c.a[ti][tj][e] = *(in ? cp[ti][tj][e] : F.at(rI, rJ));
      }
  typename TL::Acc x;
  TL::zero(x);
  TL::mma_global(F.L + (int64_t)k0 * nf + rI, nf, nf - rI, Dt, TB, w, x, lane, wave);
  E* Lf = Fbuf + t.loff[v];
  __syncthreads();   // ps
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = TL::row(lane, wave, ti, e), cl = TL::col(lane, wave, tj);
        const E val = x.a[ti][tj][e];
        Xi[r * LDT + cl] = val * ps[cl];
        if (I == J) {
          Xj[cl * LDT + r] = val;
          if (rI + r < nf && cl < w) Lf[(int64_t)(k0 + cl) * nf + rI + r] = val * ps[cl];
        }
      }
  if (I != J) {
    typename TL::Acc y;
    TL::zero(y);
    TL::mma_global(F.L + (int64_t)k0 * nf + rJ, nf, nf - rJ, Dt, TB, w, y, lane, wave);
#pragma unroll
    for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          Xj[TL::col(lane, wave, tj) * LDT + TL::row(lane, wave, ti, e)] = y.a[ti][tj][e];
  }
  __syncthreads();
  TL::mma(Xi, Xj, w, c, lane, wave, E(-1));
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (cp[ti][tj][e] != nullptr) *cp[ti][tj][e] = c.a[ti][tj][e];
}

// ---------------------------------------------------------------------------------
// Nonsymmetric fronts (a damping matrix with a skew part makes Q(sigma)
// nonsymmetric; its symmetric part sigma^2 M + sigma C_sym + K stays positive
// definite, so Gaussian elimination without pivoting has positive pivots).
// A front is kept as two lower triangles at the same offsets: the front of A
// (Lbuf / Ubuf) and the front of A^T (Rbuf / URbuf).  The factorisation is
// A = L Ut^T with L and Ut lower triangular sharing the diagonal sqrt(a_cc):
// per pivot c,  d = sqrt(a_cc),  l_rc = a_rc / d,  ut_rc = a_cr / d,  and the
// Schur complement a_rj -= l_rc ut_jc in both triangles (in the front of A^T:
// a_jr -= ut_rc l_jc).  Every kernel of the Cholesky path then runs on each
// side with the other side's panel as its second operand: the forward sweep
// uses F of L, the backward sweep F of Ut.

// Inverse of the lower block S (64 x 64 in LDS, reciprocal diagonal rd) into
// Dm, blocked by 16 as in k_potrf_diag (diagonal blocks by forward
// substitution, one wave each; the blocks below, block column by block
// column).  Called by every thread; Dm must be zero on entry.
template <class E>
__device__ __forceinline__ void lower_inverse(E (*S)[LDT], const E* rd, E (*Dm)[LDT], E (*Tx)[16][17], int lane,
                                              int wave) {
  if (lane < 16) {
    const int base = 16 * wave, c = lane;
    E dc[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      E sum = E(0);
#pragma unroll
      for (int k = 0; k < rr; ++k) sum += S[base + rr][base + k] * dc[k];
      const E ri = rd[base + rr];
      dc[rr] = (rr < c) ? E(0) : (rr == c ? ri : -sum * ri);
      Dm[base + rr][base + c] = dc[rr];
    }
  }
  __syncthreads();
  if (wave < 3) {
    const int j = wave, c = lane & 15, rg = lane >> 4;
    for (int i = j + 1; i < 4; ++i) {
      E tv[4] = {E(0), E(0), E(0), E(0)};
      for (int k = 16 * j; k < 16 * i; ++k) {
        const E dk = Dm[k][16 * j + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) tv[u] += S[16 * i + 4 * rg + u][k] * dk;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) Tx[j][4 * rg + u][c] = tv[u];
      wave_sync();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = 4 * rg + u;
        E s = E(0);
#pragma unroll
        for (int q = 0; q < 16; ++q) s += Dm[16 * i + r][16 * i + q] * Tx[j][q][c];
        Dm[16 * i + r][16 * j + c] = -s;
      }
      wave_sync();
    }
  }
  __syncthreads();
}

// LU of the diagonal block [k0, k0 + w): L_kk into Lfac, Ut_kk into Rfac,
// their inverses stored transposed at DLbuf / DUbuf (layout of k_potrf_diag).
// A pivot that is not positive (or NaN) is recorded in *status (the front's
// dof, first one wins) and replaced by 1 so that the kernel completes.
template <class E>
__global__ __launch_bounds__(FT) void k_getrf_diag(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                   const E* __restrict__ Lbuf, const E* __restrict__ Rbuf,
                                                   E* __restrict__ Lfac, E* __restrict__ Rfac,
                                                   E* __restrict__ DLbuf, E* __restrict__ DUbuf,
                                                   int64_t* __restrict__ status) {
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v];
  if (no <= k0) return;
  const int w = min(TB, no - k0);
  const E* LA = Lbuf + t.loff[v];
  const E* RA = Rbuf + t.loff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E SL[TB][LDT];
  __shared__ E SR[TB][LDT];
  __shared__ E Dm[TB][LDT];
  __shared__ E Tx[3][16][17];
  __shared__ E rd[TB];
  {
    constexpr int U = TB * TB / FT;
    E xl[U], xr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = tid + u * FT, r = idx % TB, c = idx / TB;
      const bool in = c <= r && r < w;
      const int64_t o = in ? (int64_t)(k0 + c) * nf + k0 + r : (int64_t)k0 * nf + k0;
      xl[u] = LA[o];
      xr[u] = RA[o];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = tid + u * FT, r = idx % TB, c = idx / TB;
      const bool in = c <= r && r < w;
      const E pad = (c == r && r >= w) ? E(1) : E(0);
      SL[r][c] = in ? xl[u] : pad;
      SR[r][c] = in ? xr[u] : pad;
      Dm[r][c] = E(0);
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < TB; c0 += 16) {
    if (wave == 0) {
      const int r = lane;
      E rl[16], rr_[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        rl[j] = SL[r][c0 + j];
        rr_[j] = SR[r][c0 + j];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int cc = c0 + c;
        E piv = lane_value(rl[c], cc);
        if (!(piv > E(0))) {
          if (r == cc && cc < w)
            atomicCAS((unsigned long long*)status, (unsigned long long)(-1ll),
                      (unsigned long long)t.fdofs[t.foff[v] + k0 + cc]);
          piv = E(1);
        }
        const E inv = rsqrt_refined(piv);
        const E d = piv * inv;
        if (r == cc) rd[cc] = inv;
        const E l = rl[c] * inv, u = rr_[c] * inv;   // l_r,cc and ut_r,cc (rows below the pivot)
        rl[c] = (r == cc) ? d : l;
        rr_[c] = (r == cc) ? d : u;
        if (r >= cc) {
          SL[r][cc] = rl[c];
          SR[r][cc] = rr_[c];
        }
        wave_sync();
#pragma unroll
        for (int j = c + 1; j < 16; ++j) {
          rl[j] -= l * SR[c0 + j][cc];
          rr_[j] -= u * SL[c0 + j][cc];
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (r >= c0 + j) {
          SL[r][c0 + j] = rl[j];
          SR[r][c0 + j] = rr_[j];
        }
    }
    __syncthreads();
    const int n = TB - c0 - 16;
    for (int idx = tid; idx < n * n; idx += FT) {
      const int i = idx / n, j = idx % n;
      if (j <= i) {
        const int ri = c0 + 16 + i, rj = c0 + 16 + j;
        E a = SL[ri][rj], b = SR[ri][rj];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          a -= SL[ri][c0 + c] * SR[rj][c0 + c];
          b -= SR[ri][c0 + c] * SL[rj][c0 + c];
        }
        SL[ri][rj] = a;
        SR[ri][rj] = b;
      }
    }
    __syncthreads();
  }
  E* Lf = Lfac + t.loff[v];
  E* Rf = Rfac + t.loff[v];
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int r = idx % TB, c = idx / TB;
    if (r < w && c <= r) {
      Lf[(int64_t)(k0 + c) * nf + k0 + r] = SL[r][c];
      Rf[(int64_t)(k0 + c) * nf + k0 + r] = SR[r][c];
    }
  }
  const int64_t dblk = ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  lower_inverse<E>(SL, rd, Dm, Tx, lane, wave);
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int c = idx / TB, r = idx % TB;
    DLbuf[dblk + idx] = (r < w && c < w) ? Dm[r][c] : E(0);
  }
  __syncthreads();
  for (int idx = tid; idx < TB * TB; idx += FT) Dm[idx / TB][idx % TB] = E(0);
  __syncthreads();
  lower_inverse<E>(SR, rd, Dm, Tx, lane, wave);
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int c = idx / TB, r = idx % TB;
    DUbuf[dblk + idx] = (r < w && c < w) ? Dm[r][c] : E(0);
  }
}

// Panel rows and trailing updates of both triangles below the panel
// [k0, k0 + w), one workgroup per tile pair (I, J), J <= I (as
// k_panel_update): X = A_panel D_U^T (rows of L), Y = At_panel D_L^T (rows of
// Ut), C^A_IJ -= X_I Y_J^T on the front of A and C^At_IJ -= Y_I X_J^T on the
// front of A^T; the diagonal pair writes X_I and Y_I as factor rows.
template <class E>
__global__ __launch_bounds__(FT) void k_panel_update_lu(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                        E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                        E* __restrict__ Rbuf, E* __restrict__ URbuf,
                                                        E* __restrict__ Lfac, E* __restrict__ Rfac,
                                                        const E* __restrict__ DLbuf, const E* __restrict__ DUbuf) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> FA = front_of(t, v, Lbuf, Ubuf);
  const Front<E> FT_ = front_of(t, v, Rbuf, URbuf);
  if (FA.no <= k0) return;
  const int w = min(TB, FA.no - k0);
  const int s0 = k0 + w;
  const int pidx = blockIdx.y;
  int I = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= pidx) ++I;
  while (I * (I + 1) / 2 > pidx) --I;
  const int J = pidx - I * (I + 1) / 2;
  const int rI = s0 + TB * I, rJ = s0 + TB * J;
  if (rI >= FA.nf) return;
  const int nf = FA.nf;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E Xa[TB * LDT];   // A operand (row panel of one side)
  __shared__ E Xb[TB * LDT];   // B operand (transposed row panel of the other side)
  const int64_t dblk = ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  const E* DtL = DLbuf + dblk;
  const E* DtU = DUbuf + dblk;
  E* Lf = Lfac + t.loff[v];
  E* Rf = Rfac + t.loff[v];
  // the C tiles' current values of both sides, loaded before the products
  typename TL::Acc ca, ct;
  E* pa[TL::TI][TL::TJ][4];
  E* pt[TL::TI][TL::TJ][4];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rI + TL::row(lane, wave, ti, e), cc = rJ + TL::col(lane, wave, tj);
        const bool in = r < nf && cc < nf && r >= cc;
        pa[ti][tj][e] = in ? FA.at(r, cc) : nullptr;
        pt[ti][tj][e] = in ? FT_.at(r, cc) : nullptr;
        ca.a[ti][tj][e] = *(in ? pa[ti][tj][e] : FA.at(rI, rJ));
        ct.a[ti][tj][e] = *(in ? pt[ti][tj][e] : FT_.at(rI, rJ));
      }
  typename TL::Acc xi, yi, xj, yj;
  TL::zero(xi);
  TL::zero(yi);
  TL::mma_global(FA.L + (int64_t)k0 * nf + rI, nf, nf - rI, DtU, TB, w, xi, lane, wave);
  TL::mma_global(FT_.L + (int64_t)k0 * nf + rI, nf, nf - rI, DtL, TB, w, yi, lane, wave);
  if (I != J) {
    TL::zero(xj);
    TL::zero(yj);
    TL::mma_global(FA.L + (int64_t)k0 * nf + rJ, nf, nf - rJ, DtU, TB, w, xj, lane, wave);
    TL::mma_global(FT_.L + (int64_t)k0 * nf + rJ, nf, nf - rJ, DtL, TB, w, yj, lane, wave);
  }
  // front of A: C -= X_I Y_J^T
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = TL::row(lane, wave, ti, e), cl = TL::col(lane, wave, tj);
        const E xv = xi.a[ti][tj][e], yv = (I == J) ? yi.a[ti][tj][e] : yj.a[ti][tj][e];
        Xa[r * LDT + cl] = xv;
        Xb[cl * LDT + r] = yv;
        if (I == J && rI + r < nf && cl < w) {
          Lf[(int64_t)(k0 + cl) * nf + rI + r] = xv;
          Rf[(int64_t)(k0 + cl) * nf + rI + r] = yi.a[ti][tj][e];
        }
      }
  __syncthreads();
  TL::mma(Xa, Xb, w, ca, lane, wave, E(-1));
  __syncthreads();
  // front of A^T: C -= Y_I X_J^T
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = TL::row(lane, wave, ti, e), cl = TL::col(lane, wave, tj);
        Xa[r * LDT + cl] = yi.a[ti][tj][e];
        Xb[cl * LDT + r] = (I == J) ? xi.a[ti][tj][e] : xj.a[ti][tj][e];
      }
  __syncthreads();
  TL::mma(Xa, Xb, w, ct, lane, wave, E(-1));
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (pa[ti][tj][e] != nullptr) {
          *pa[ti][tj][e] = ca.a[ti][tj][e];
          *pt[ti][tj][e] = ct.a[ti][tj][e];
        }
}

// Large symmetric fronts in two launches per panel (as for the LU fronts
// below): k_panel_rows forms X_I = A_panel D^T once per row tile and stores
// the factor rows X_I S; k_panel_trail updates each tile pair from them read
// straight from the factor, C_IJ -= (X_I S) (X_J S)^T S (S = diag of the
// pivot signs, S^2 = I).
template <class E>
__global__ __launch_bounds__(FT) void k_panel_rows(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                   E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                   E* __restrict__ Fbuf, const E* __restrict__ Dbuf) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  if (F.no <= k0) return;
  const int w = min(TB, F.no - k0);
  const int rI = k0 + w + TB * (int)blockIdx.y;
  const int nf = F.nf;
  if (rI >= nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E ps[TB];
  if (tid < TB) ps[tid] = (t.sgn != nullptr && tid < w) ? (E)t.sgn[t.fdofs[t.foff[v] + k0 + tid]] : E(1);
  const E* Dt = Dbuf + ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  typename TL::Acc x;
  TL::zero(x);
  TL::mma_global(F.L + (int64_t)k0 * nf + rI, nf, nf - rI, Dt, TB, w, x, lane, wave);
  __syncthreads();   // ps
  E* Lf = Fbuf + t.loff[v];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = TL::row(lane, wave, ti, e), cl = TL::col(lane, wave, tj);
        if (rI + r < nf && cl < w) Lf[(int64_t)(k0 + cl) * nf + rI + r] = x.a[ti][tj][e] * ps[cl];
      }
}

template <class E>
__global__ __launch_bounds__(FT) void k_panel_trail(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                    E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                    const E* __restrict__ Fbuf) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  if (F.no <= k0) return;
  const int w = min(TB, F.no - k0);
  const int s0 = k0 + w;
  const int pidx = blockIdx.y;
  int I = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= pidx) ++I;
  while (I * (I + 1) / 2 > pidx) --I;
  const int J = pidx - I * (I + 1) / 2;
  const int rI = s0 + TB * I, rJ = s0 + TB * J;
  const int nf = F.nf;
  if (rI >= nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E ps[TB];
  if (tid < TB) ps[tid] = (t.sgn != nullptr && tid < w) ? (E)t.sgn[t.fdofs[t.foff[v] + k0 + tid]] : E(1);
  typename TL::Acc c;
  E* cp[TL::TI][TL::TJ][4];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rI + TL::row(lane, wave, ti, e), cc = rJ + TL::col(lane, wave, tj);
        const bool in = r < nf && cc < nf && r >= cc;
        cp[ti][tj][e] = in ? F.at(r, cc) : nullptr;
        c.a[ti][tj][e] = *(in ? cp[ti][tj][e] : F.at(rI, rJ));
      }
  const E* Lf = Fbuf + t.loff[v];
  __syncthreads();   // ps
  typename TL::Acc pr;
  TL::zero(pr);
  TL::mma_global_nt(Lf + (int64_t)k0 * nf + rI, nf, nf - rI, Lf + (int64_t)k0 * nf + rJ, nf, nf - rJ, w, pr, lane,
                    wave, t.sgn != nullptr ? ps : nullptr);
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (cp[ti][tj][e] != nullptr) *cp[ti][tj][e] = c.a[ti][tj][e] - pr.a[ti][tj][e];
}

// Large LU fronts in two launches per panel, so that no panel row is formed
// twice (the fused kernel above forms X_I, Y_I and X_J, Y_J for every tile
// pair, i.e. each row tile once per pair it takes part in):
// k_panel_rows_lu, one workgroup per row tile I below the panel: X_I =
// A_panel D_U^T and Y_I = At_panel D_L^T written as factor rows;
// k_panel_trail_lu, one workgroup per tile pair (I, J), J <= I: the stored
// rows read straight from the factor, C^A_IJ -= X_I Y_J^T and
// C^At_IJ -= Y_I X_J^T.
template <class E>
__global__ __launch_bounds__(FT) void k_panel_rows_lu(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                      E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                      E* __restrict__ Rbuf, E* __restrict__ URbuf,
                                                      E* __restrict__ Lfac, E* __restrict__ Rfac,
                                                      const E* __restrict__ DLbuf, const E* __restrict__ DUbuf) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> FA = front_of(t, v, Lbuf, Ubuf);
  const Front<E> FT_ = front_of(t, v, Rbuf, URbuf);
  if (FA.no <= k0) return;
  const int w = min(TB, FA.no - k0);
  const int rI = k0 + w + TB * (int)blockIdx.y;
  const int nf = FA.nf;
  if (rI >= nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t dblk = ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  typename TL::Acc xi, yi;
  TL::zero(xi);
  TL::zero(yi);
  TL::mma_global(FA.L + (int64_t)k0 * nf + rI, nf, nf - rI, DUbuf + dblk, TB, w, xi, lane, wave);
  TL::mma_global(FT_.L + (int64_t)k0 * nf + rI, nf, nf - rI, DLbuf + dblk, TB, w, yi, lane, wave);
  E* Lf = Lfac + t.loff[v];
  E* Rf = Rfac + t.loff[v];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = TL::row(lane, wave, ti, e), cl = TL::col(lane, wave, tj);
        if (rI + r < nf && cl < w) {
          Lf[(int64_t)(k0 + cl) * nf + rI + r] = xi.a[ti][tj][e];
          Rf[(int64_t)(k0 + cl) * nf + rI + r] = yi.a[ti][tj][e];
        }
      }
}

template <class E>
__global__ __launch_bounds__(FT) void k_panel_trail_lu(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                       E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                       E* __restrict__ Rbuf, E* __restrict__ URbuf,
                                                       const E* __restrict__ Lfac, const E* __restrict__ Rfac) {
  typedef Tile64<E, 4> TL;
  const int v = level_nodes[blockIdx.x];
  const Front<E> FA = front_of(t, v, Lbuf, Ubuf);
  const Front<E> FT_ = front_of(t, v, Rbuf, URbuf);
  if (FA.no <= k0) return;
  const int w = min(TB, FA.no - k0);
  const int s0 = k0 + w;
  const int pidx = blockIdx.y;
  int I = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= pidx) ++I;
  while (I * (I + 1) / 2 > pidx) --I;
  const int J = pidx - I * (I + 1) / 2;
  const int rI = s0 + TB * I, rJ = s0 + TB * J;
  const int nf = FA.nf;
  if (rI >= nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const E* Lf = Lfac + t.loff[v];
  const E* Rf = Rfac + t.loff[v];
  typename TL::Acc ca, ct;
  E* pa[TL::TI][TL::TJ][4];
  E* pt[TL::TI][TL::TJ][4];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rI + TL::row(lane, wave, ti, e), cc = rJ + TL::col(lane, wave, tj);
        const bool in = r < nf && cc < nf && r >= cc;
        pa[ti][tj][e] = in ? FA.at(r, cc) : nullptr;
        pt[ti][tj][e] = in ? FT_.at(r, cc) : nullptr;
        ca.a[ti][tj][e] = *(in ? pa[ti][tj][e] : FA.at(rI, rJ));
        ct.a[ti][tj][e] = *(in ? pt[ti][tj][e] : FT_.at(rI, rJ));
      }
  // C^A -= X_I Y_J^T and C^At -= Y_I X_J^T with the stored rows read straight
  // from the factor (no staging: no LDS, more workgroups per compute unit)
  typename TL::Acc pr;
  TL::zero(pr);
  TL::mma_global_nt(Lf + (int64_t)k0 * nf + rI, nf, nf - rI, Rf + (int64_t)k0 * nf + rJ, nf, nf - rJ, w, pr, lane,
                    wave);
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) ca.a[ti][tj][e] -= pr.a[ti][tj][e];
  TL::zero(pr);
  TL::mma_global_nt(Rf + (int64_t)k0 * nf + rI, nf, nf - rI, Lf + (int64_t)k0 * nf + rJ, nf, nf - rJ, w, pr, lane,
                    wave);
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) ct.a[ti][tj][e] -= pr.a[ti][tj][e];
#pragma unroll
  for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (pa[ti][tj][e] != nullptr) {
          *pa[ti][tj][e] = ca.a[ti][tj][e];
          *pt[ti][tj][e] = ct.a[ti][tj][e];
        }
}

// Rows [64 y, +64) of X with X L_oo = [I; L_bo] (L from the factor buffer);
// X row r at Fout[r * no + ...] (the front buffer's block of the node).
// Sixteen waves: each takes one 16 x 16 MFMA tile of a 64 x 64 product.
constexpr int RT_THREADS = 1024;
template <class E>
__global__ __launch_bounds__(RT_THREADS) void k_rtrsm(DevTree t, const int* __restrict__ level_nodes,
                                                      const E* __restrict__ Lfac, E* __restrict__ Fout,
                                                      const E* __restrict__ Dbuf) {
  typedef Tile64<E, RT_THREADS / 64> TL;
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v];
  const int r0 = TB * blockIdx.y;
  if (r0 >= nf || no == 0) return;
  const E* L = Lfac + t.loff[v];
  E* T = Fout + t.loff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E As[TB * LDT];
  __shared__ E Bs[TB * LDT];
  const int npan = (no + TB - 1) / TB;
  const bool top = (r0 + TB <= no);            // every row of the block is an own row
  for (int P = npan - 1; P >= 0; --P) {
    const int c0 = P * TB, w = min(TB, no - c0);
    if (top && r0 + TB - 1 < c0) {               // X[r][c] = 0 for c > r < no
      for (int idx = tid; idx < TB * TB; idx += RT_THREADS) {
        const int i = idx / TB, j = idx % TB;
        if (j < w) T[(int64_t)(r0 + i) * no + c0 + j] = E(0);
      }
      continue;
    }
    typename TL::Acc acc;
#pragma unroll
    for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + TL::row(lane, wave, ti, e), c = c0 + TL::col(lane, wave, tj);
          const bool bnd = r < nf && c < c0 + w && r >= no;
          const E lv = L[bnd ? (int64_t)c * nf + r : 0];
          acc.a[ti][tj][e] = bnd ? lv : ((r < nf && c < c0 + w && r == c) ? E(1) : E(0));
        }
    // minus X[:, kb] L[kb, P] over solved block columns kb > P (X vanishes past the diagonal for top rows)
    const int kbmax = top ? min(npan - 1, (r0 + TB - 1) / TB) : npan - 1;
    for (int kb = P + 1; kb <= kbmax; ++kb) {
      const int cb = kb * TB, wb = min(TB, no - cb);
      // every load of both tiles issued before the first LDS store
      constexpr int U = TB * TB / RT_THREADS;
      E xa[U], xb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = tid + u * RT_THREADS, k = idx % TB, i = idx / TB;
        const bool ina = r0 + i < nf && k < wb;   // As[i][k] = X[r0 + i][cb + k], coalesced in k
        const bool inb = k < wb && i < w;          // Bs[k][i] = L[cb + k][c0 + i], coalesced in k
        xa[u] = T[ina ? (int64_t)(r0 + i) * no + cb + k : 0];
        xb[u] = L[inb ? (int64_t)(c0 + i) * nf + cb + k : 0];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = tid + u * RT_THREADS, k = idx % TB, i = idx / TB;
        As[i * LDT + k] = (r0 + i < nf && k < wb) ? xa[u] : E(0);
        Bs[k * LDT + i] = (k < wb && i < w) ? xb[u] : E(0);
      }
      __syncthreads();
      TL::mma(As, Bs, wb, acc, lane, wave, E(-1));
    }
    // X[:, P] = acc D_P
    __syncthreads();
    // D_P (stored transposed: Dt[j * 64 + k] = D[k][j]) as the B operand
    const E* Dt = Dbuf + ((int64_t)t.doff[v] + P) * (TB * TB);
    {
      constexpr int U = TB * TB / RT_THREADS;
      E xd[U];
#pragma unroll
      for (int u = 0; u < U; ++u) xd[u] = Dt[tid + u * RT_THREADS];
#pragma unroll
      for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            As[TL::row(lane, wave, ti, e) * LDT + TL::col(lane, wave, tj)] = acc.a[ti][tj][e];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = tid + u * RT_THREADS;
        Bs[(idx % TB) * LDT + idx / TB] = xd[u];
      }
    }
    __syncthreads();
    typename TL::Acc x;
    TL::zero(x);
    TL::mma(As, Bs, w, x, lane, wave, E(1));
#pragma unroll
    for (int ti = 0; ti < TL::TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TL::TJ; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + TL::row(lane, wave, ti, e), c = TL::col(lane, wave, tj);
          if (r < nf && c < w) T[(int64_t)r * no + c0 + c] = x.a[ti][tj][e];
        }
    __syncthreads();   // T of this block column is read as the next panel's A operand
  }
}

// Sweep layouts of F (rows of T, F[r][c] at T[r * no + c]) with K = 16 bytes /
// element consecutive entries side by side, so that one lane reads K of them
// with a single 16-byte load (kernels.hpp: lp_group, tp_group):
//   Lp: columns in groups of K, F[r][gK + s] at Lp[(lp_group(g) + r - gK) K + s]
//       for r >= gK, g < ceil(no/K) (forward sweep: lane = row);
//   Tp: rows in groups of K, F[gK + s][a] at Tp[(tp_group(g) + a) K + s] for
//       a < tp_width(g), g < ceil(nf/K) (backward sweep: lane = own column a),
//       or at Tp[(g no + a) K + s] for every a < no where t.ttri marks the node
//       as keeping the full rectangle.
// The entries left out are the zeros of L_oo^{-1} above its diagonal blocks of
// K; padding columns / rows are written as zeros.  64 x 64 tiles through LDS.
// (For an LU factor the forward layout comes from F of L and the backward one
// from F of Ut, the transposed upper factor: TbufT; TbufT = Tbuf otherwise.)
template <class E>
__global__ __launch_bounds__(FT) void k_pack(DevTree t, const int* __restrict__ level_nodes,
                                             const E* __restrict__ Tbuf, const E* __restrict__ TbufT,
                                             E* __restrict__ Lp, E* __restrict__ Tp) {
  constexpr int K = 16 / sizeof(E);
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v];
  const int nfp = (nf + K - 1) / K * K, nop = (no + K - 1) / K * K;
  const int ntr = (nfp + TB - 1) / TB;
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  const int r0 = tr * TB, c0 = tc * TB;
  if (r0 >= nfp || c0 >= nop) return;
  __shared__ E S[TB * LDT];
  auto stage = [&](const E* __restrict__ T) {
    constexpr int U = TB * TB / FT;
    E x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = threadIdx.x + u * FT, i = idx / TB, c = idx % TB;   // row r0 + i, contiguous in c
      const bool in = r0 + i < nf && c0 + c < no;
      x[u] = T[in ? (int64_t)(r0 + i) * no + c0 + c : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = threadIdx.x + u * FT, i = idx / TB, c = idx % TB;
      S[i * LDT + c] = (r0 + i < nf && c0 + c < no) ? x[u] : E(0);
    }
  };
  stage(Tbuf + t.loff[v]);
  __syncthreads();
  E* L = Lp + t.lpoff[v];
  for (int idx = threadIdx.x; idx < TB * TB; idx += FT) {
    const int gl = idx / (TB * K), rem = idx % (TB * K), r = rem / K, sl = rem % K;
    const int c = gl * K + sl;
    const int rr = r0 + r, g = (c0 + c) / K;
    if (rr < nf && c0 + c < nop && rr >= g * K) L[(lp_group(g, nf, K) + rr - g * K) * K + sl] = S[r * LDT + c];
  }
  if (TbufT != Tbuf) {
    __syncthreads();
    stage(TbufT + t.loff[v]);
    __syncthreads();
  }
  E* Tq = Tp + t.tpoff[v];
  const bool tri = t.ttri[v] != 0;
  for (int idx = threadIdx.x; idx < TB * TB; idx += FT) {
    const int gl = idx / (TB * K), rem = idx % (TB * K), c = rem / K, sl = rem % K;
    const int r = gl * K + sl;
    const int g = (r0 + r) / K, cc = c0 + c;
    if (tri) {
      if (r0 + r < nfp && cc < tp_width(g, no, K)) Tq[(tp_group(g, no, K) + cc) * K + sl] = S[r * LDT + c];
    } else {
      if (r0 + r < nfp && cc < no) Tq[((int64_t)g * no + cc) * K + sl] = S[r * LDT + c];
    }
  }
}
// One tree level.  Lf: the front buffer (assembled front, updated in place;
// receives F), Lx: the factor buffer (L), U: update blocks, D: diagonal-block
// inverses.
template <class E>
void front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                  int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                  const double* C, E* Lf, E* U, E* Lx, E* D, E* Lp, E* Tp, const float* U32,
                  const double* U64, int64_t* status, hipStream_t st) {
  if (count <= 0) return;
  const int ncol = (max_nf + TB - 1) / TB;
  hipLaunchKernelGGL(k_front_assemble<E>, dim3(count, ncol), dim3(FT), (size_t)2 * max_nf * sizeof(int), st, s.n,
                     s.lo, s.hi, s.rowptr, s.col, t, level_nodes, s2, s1, K, M, C, Lf, U);
  if (max_child_nb > 0)
    for (int slot = 0; slot < max_kids; ++slot)
      hipLaunchKernelGGL(k_front_extend<E>, dim3(count, (max_child_nb + TB - 1) / TB), dim3(FT),
                         (size_t)max_child_nb * sizeof(int), st, t,
                         level_nodes, slot, Lf, U, U32, U64);
  for (int k0 = 0; k0 < max_no; k0 += TB) {
    hipLaunchKernelGGL(k_potrf_diag<E>, dim3(count), dim3(FT), 0, st, t, level_nodes, k0, (const E*)Lf, Lx, D,
                       status, (unsigned long long*)(status + 1));
    // row tiles below a block that is at least one column wide; one workgroup per tile pair
    const int below = std::max(1, max_nf - k0 - 1);
    const int nrc = (below + TB - 1) / TB;
    if (split_panel(count, nrc)) {
      hipLaunchKernelGGL(k_panel_rows<E>, dim3(count, nrc), dim3(FT), 0, st, t, level_nodes, k0, Lf, U, Lx,
                         (const E*)D);
      hipLaunchKernelGGL(k_panel_trail<E>, dim3(count, nrc * (nrc + 1) / 2), dim3(FT), 0, st, t, level_nodes, k0,
                         Lf, U, (const E*)Lx);
    } else {
      hipLaunchKernelGGL(k_panel_update<E>, dim3(count, nrc * (nrc + 1) / 2), dim3(FT), 0, st, t, level_nodes, k0,
                         Lf, U, Lx, (const E*)D);
    }
  }
  const int nrt = (max_nf + TB - 1) / TB;
  hipLaunchKernelGGL(k_rtrsm<E>, dim3(count, nrt), dim3(RT_THREADS), 0, st, t, level_nodes, (const E*)Lx, Lf,
                     (const E*)D);
  const int nct = (max_no + 3 + TB - 1) / TB, nrp = (max_nf + 3 + TB - 1) / TB;
  hipLaunchKernelGGL(k_pack<E>, dim3(count, nrp * nct), dim3(FT), 0, st, t, level_nodes, (const E*)Lf, (const E*)Lf,
                     Lp, Tp);
}

void launch_front_factor_lu(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                            int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K,
                            const double* M, const double* C, const double* Ct, double* L, double* U, double* Lx,
                            double* D, double* R, double* UR, double* Rx, double* DR, double* Lp, double* Tp,
                            int64_t* status, hipStream_t st) {
  if (count <= 0) return;
  typedef double E;
  const int ncol = (max_nf + TB - 1) / TB;
  // a front holds the transpose of the rows it is assembled from: the front
  // of A takes the rows of A^T (C^T values), the front of A^T those of A
  hipLaunchKernelGGL(k_front_assemble<E>, dim3(count, ncol), dim3(FT), (size_t)2 * max_nf * sizeof(int), st, s.n,
                     s.lo, s.hi, s.rowptr, s.col, t, level_nodes, s2, s1, K, M, Ct, L, U);
  hipLaunchKernelGGL(k_front_assemble<E>, dim3(count, ncol), dim3(FT), (size_t)2 * max_nf * sizeof(int), st, s.n,
                     s.lo, s.hi, s.rowptr, s.col, t, level_nodes, s2, s1, K, M, C, R, UR);
  if (max_child_nb > 0)
    for (int slot = 0; slot < max_kids; ++slot) {
      hipLaunchKernelGGL(k_front_extend<E>, dim3(count, (max_child_nb + TB - 1) / TB), dim3(FT),
                         (size_t)max_child_nb * sizeof(int), st, t, level_nodes, slot, L, U, (const float*)nullptr,
                         (const double*)U);
      hipLaunchKernelGGL(k_front_extend<E>, dim3(count, (max_child_nb + TB - 1) / TB), dim3(FT),
                         (size_t)max_child_nb * sizeof(int), st, t, level_nodes, slot, R, UR, (const float*)nullptr,
                         (const double*)UR);
    }
  for (int k0 = 0; k0 < max_no; k0 += TB) {
    hipLaunchKernelGGL(k_getrf_diag<E>, dim3(count), dim3(FT), 0, st, t, level_nodes, k0, (const E*)L, (const E*)R,
                       Lx, Rx, D, DR, status);
    const int below = std::max(1, max_nf - k0 - 1);
    const int nrc = (below + TB - 1) / TB;
    if (split_panel(count, nrc)) {
      hipLaunchKernelGGL(k_panel_rows_lu<E>, dim3(count, nrc), dim3(FT), 0, st, t, level_nodes, k0, L, U, R, UR, Lx,
                         Rx, (const E*)D, (const E*)DR);
      hipLaunchKernelGGL(k_panel_trail_lu<E>, dim3(count, nrc * (nrc + 1) / 2), dim3(FT), 0, st, t, level_nodes, k0,
                         L, U, R, UR, (const E*)Lx, (const E*)Rx);
    } else {
      hipLaunchKernelGGL(k_panel_update_lu<E>, dim3(count, nrc * (nrc + 1) / 2), dim3(FT), 0, st, t, level_nodes,
                         k0, L, U, R, UR, Lx, Rx, (const E*)D, (const E*)DR);
    }
  }
  const int nrt = (max_nf + TB - 1) / TB;
  hipLaunchKernelGGL(k_rtrsm<E>, dim3(count, nrt), dim3(RT_THREADS), 0, st, t, level_nodes, (const E*)Lx, L,
                     (const E*)D);
  hipLaunchKernelGGL(k_rtrsm<E>, dim3(count, nrt), dim3(RT_THREADS), 0, st, t, level_nodes, (const E*)Rx, R,
                     (const E*)DR);
  const int nct = (max_no + 3 + TB - 1) / TB, nrp = (max_nf + 3 + TB - 1) / TB;
  hipLaunchKernelGGL(k_pack<E>, dim3(count, nrp * nct), dim3(FT), 0, st, t, level_nodes, (const E*)L, (const E*)R,
                     Lp, Tp);
}

void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                         int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                         const double* C, double* L, double* U, double* T, double* D, double* Lp, double* Tp,
                         const float* U32, int64_t* status, hipStream_t st) {
  front_factor<double>(s, t, level_nodes, count, max_no, max_nf, max_child_nb, max_kids, s2, s1, K, M, C, L, U, T, D, Lp, Tp,
                       U32, U, status, st);
}

void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                         int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                         const double* C, float* L, float* U, float* T, float* D, float* Lp, float* Tp,
                         int64_t* status, hipStream_t st) {
  // FP32 fronts only have FP32 children
  front_factor<float>(s, t, level_nodes, count, max_no, max_nf, max_child_nb, max_kids, s2, s1, K, M, C, L, U, T, D, Lp, Tp,
                      U, nullptr, status, st);
}

}  // namespace riga
