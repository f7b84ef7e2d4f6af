// Multifrontal Cholesky of Q(sigma) = sigma^2 M + sigma C + K over the
// nested-dissection tree (Sec. 3.3: rIGA hyperplanes are the separators;
// Sec. 5.2.1: one factorization per shift).
//
// A front of node v holds its own dofs (eliminated here) followed by its
// boundary dofs (ancestors coupled to the subtree).  Storage per node:
//   L block  nf x no, column-major (ld nf): the own columns of the front;
//   U block  nb x nb, column-major: the update (Schur complement) matrix that
//            the parent adds into its front ("extend-add");
//   T block  no x nf, column-major (same offset as L): F^T, the rows of F.
// A tree level is processed by a pipeline of batched kernels whose grids span
// every node of the level:
//   k_front_assemble   zero the front and add the original entries of Q
//                      (64 front columns per workgroup);
//   k_front_extend     add the children's update blocks, one child slot per
//                      launch (64 child columns per workgroup);
//   per 64-wide panel of own columns:
//     k_potrf_diag     Cholesky of the 64x64 diagonal block and its inverse
//                      D_k = L_kk^{-1} (one workgroup per node, in LDS);
//     k_trsm_panel     panel rows below the block: X = A D_k^T   (MFMA)
//     k_syrk_update    trailing lower triangle, own and update parts:
//                      C -= P_I P_J^T on 64x64 tiles             (MFMA)
//   k_rtrsm            rows of F = [L_oo^{-1}; L_bo L_oo^{-1}] from
//                      X L_oo = [I; L_bo], block column by block column from
//                      the right with the stored D_k               (MFMA)
//   k_pack             F in the two sweep layouts Lp / Tp (16-byte groups of
//                      columns / rows).
// With F, each forward/backward sweep is one matrix-vector product per node.
// Every kernel is a template over the element type E of the node's front:
// double (v_mfma_f64_16x16x4_f64) or float (v_mfma_f32_16x16x4_f32, FP32
// products and accumulation) for the mixed-precision factorization, where the
// lower tree levels are FP32 and the top levels FP64.  Products run on 64x64
// tiles staged in LDS; each of the four waves owns a 32x32 quadrant (2x2 MFMA
// tiles).
#include "kernels.hpp"
#include "mfma_layout.hpp"

#include <algorithm>

namespace riga {

constexpr int FT = 256;     // threads per workgroup
constexpr int TB = 64;      // panel / tile width
constexpr int LDT = TB + 1; // LDS row stride (elements)

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

// acc += sign * A (64 x kw) B (kw x 64), A at As[i * LDT + k], B at Bs[k * LDT + j];
// wave w owns rows 32 (w >> 1) .. and columns 32 (w & 1) .., as 2 x 2 MFMA tiles.
template <class E>
__device__ __forceinline__ void mma64(const E* As, const E* Bs, int kw, acc_t<E> (&acc)[2][2],
                                      int lane, int wave, E sign) {
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  for (int k0 = 0; k0 < kw; k0 += 4) {
    const int k = k0 + mfma_ab_k(lane);
    E a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = (k < kw) ? sign * As[(wr + 16 * t + mfma_a_row(lane)) * LDT + k] : E(0);
      b[t] = (k < kw) ? Bs[k * LDT + wc + 16 * t + mfma_b_col(lane)] : E(0);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = Mfma<E>::mma(a[ti], b[tj], acc[ti][tj]);
  }
}

template <class E>
__device__ __forceinline__ int acc_row(int lane, int wave, int ti, int v) {
  return (wave >> 1) * 32 + 16 * ti + Mfma<E>::drow(lane, v);
}
__device__ __forceinline__ int acc_col(int lane, int wave, int tj) {
  return (wave & 1) * 32 + 16 * tj + mfma_d_col(lane);
}

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
    int n, const int* lo, const int* hi, const int64_t* rowptr,
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
    const int i = d % n, j = d / n;
    m_lx = lo[i];
    m_wx = hi[i] - m_lx + 1;
    m_ly = lo[j];
    const int64_t r0 = rowptr[d];
    m_k0 = (int)(r0 - rowptr[0]);
    m_len = (int)(rowptr[d + 1] - r0);
  }
  const int64_t kbase = rowptr[0];
  for (int u = 0; u < na; ++u) {
    const int a = c0 + wave + (FT / 64) * u;
    const int lx = __builtin_amdgcn_readlane(m_lx, u), wx = __builtin_amdgcn_readlane(m_wx, u);
    const int ly = __builtin_amdgcn_readlane(m_ly, u);
    const int64_t k0 = kbase + __builtin_amdgcn_readlane(m_k0, u);
    const int64_t k1 = k0 + __builtin_amdgcn_readlane(m_len, u);
    for (int64_t k = k0 + lane; k < k1; k += 64) {
      const int o = (int)(k - k0);
      const int g = (ly + o / wx) * n + lx + o % wx + base;
      int x0 = 0, x1 = nf;  // binary search of g among the sorted front keys
      while (x1 - x0 > 1) {
        const int c = (x0 + x1) >> 1;
        if (keys[c] <= g) x0 = c; else x1 = c;
      }
      if (keys[x0] == g) {
        const int pos = keys[nf + x0];
        if (pos >= a) F.L[(int64_t)a * nf + pos] = (E)(s2 * Mv[k] + s1 * Cv[k] + Kv[k]);
      }
    }
  }
}

// Columns [l0, l1) of a child's update block U (nbc x nbc, lower triangle)
// added into the parent front at the mapped positions (mk: the map from child
// row l0 on, in shared memory).  A lane owns rows k and walks the tile's
// columns in batches of eight: the eight front entries are distinct (the map
// is injective), so their loads are all issued before the sums are stored.
template <class E, class S>
__device__ __forceinline__ void extend_tile(const Front<E>& F, const S* __restrict__ Uc, int nbc, int l0, int l1,
                                            const int* mk) {
  for (int k = l0 + (int)threadIdx.x; k < nbc; k += FT) {
    const int pk = mk[k - l0];
    const int lend = min(l1, k + 1);
    int l = l0;
    for (; l + 8 <= lend; l += 8) {
      E* p[8];
      E f[8];
      S u[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        p[e] = F.at(pk, mk[l + e - l0]);
        u[e] = Uc[(int64_t)(l + e) * nbc + k];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) f[e] = *p[e];
#pragma unroll
      for (int e = 0; e < 8; ++e) *p[e] = f[e] + (E)u[e];
    }
    for (; l < lend; ++l) *F.at(pk, mk[l - l0]) += (E)Uc[(int64_t)l * nbc + k];
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

// Cholesky of the diagonal block [k0, k0+w) and D = its inverse (lower), stored
// at D + (doff[v] + k0/64) * 4096 as D[r * 64 + c].  One wave does both with
// the block in registers: lane = row for the factorisation (right-looking: at
// column c every lane scales its entry and updates the rest of its row from
// column c of the other rows, read across lanes), then lane = column for the
// inverse (forward substitution against the rows of L, broadcast from shared
// memory, four rows at a time, with the reciprocal pivots of the
// factorisation).  Every loop is unrolled so the row / column stays in
// registers.
template <class E>
__global__ __launch_bounds__(FT) void k_potrf_diag(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                   E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                   E* __restrict__ Dbuf,
                                                   int64_t* __restrict__ status) {
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  if (F.no <= k0) return;
  const int w = min(TB, F.no - k0);
  const int tid = threadIdx.x;
  __shared__ E S[TB][LDT];
  __shared__ E rd[TB];    // reciprocal pivots
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int r = idx % TB, c = idx / TB;       // coalesced along the column
    S[r][c] = (r < w && c <= r) ? F.L[(int64_t)(k0 + c) * F.nf + k0 + r] : E(0);
  }
  if (tid < TB) rd[tid] = E(0);
  __syncthreads();
  E* D = Dbuf + ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  if (tid < TB) {
    const int r = tid;
    E row[TB];
#pragma unroll
    for (int k = 0; k < TB; ++k) row[k] = S[r][k];
#pragma unroll
    for (int c = 0; c < TB; ++c) {
      if (c < w) {   // uniform
        E piv = lane_value(row[c], c);
        if (!(piv > E(0))) {           // not SPD (or NaN): record, continue with 1
          if (r == c)
            atomicCAS((unsigned long long*)status, (unsigned long long)(-1ll),
                      (unsigned long long)t.fdofs[t.foff[v] + k0 + c]);
          piv = E(1);
        }
        const E inv = rsqrt_refined(piv);
        const E d = piv * inv;
        if (r == c) rd[c] = inv;
        const E lrc = row[c] * inv;   // L[r][c] (rows below the pivot)
        const E tc = lrc * inv;
#pragma unroll
        for (int j = c + 1; j < TB; ++j) row[j] -= tc * lane_value(row[c], j);
        row[c] = (r == c) ? d : lrc;
      }
    }
#pragma unroll
    for (int k = 0; k < TB; ++k)
      if (k <= r) S[r][k] = row[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // inverse, lane = column c: D[rr][c] = -(sum_k L[rr][k] D[k][c]) / L[rr][rr],
    // the products over the rows already done formed for four rows together
    const int c = tid;
    E dc[TB];
#pragma unroll
    for (int r0 = 0; r0 < TB; r0 += 4) {
      E sp[4] = {E(0), E(0), E(0), E(0)};
#pragma unroll
      for (int k = 0; k < r0; ++k) {
        const E x = dc[k];
#pragma unroll
        for (int u = 0; u < 4; ++u) sp[u] += S[r0 + u][k] * x;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r0 + u;
        E sum = sp[u];
#pragma unroll
        for (int k = r0; k < rr; ++k) sum += S[rr][k] * dc[k];
        const E ri = rd[rr];
        dc[rr] = (rr < c) ? E(0) : (rr == c ? ri : -sum * ri);
        D[rr * TB + c] = dc[rr];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int r = idx % TB, c = idx / TB;
    if (r < w && c <= r) F.L[(int64_t)(k0 + c) * F.nf + k0 + r] = S[r][c];
  }
}

// Panel rows [k0 + w + 64 y, +64) of columns [k0, k0 + w): X = A D^T.
template <class E>
__global__ __launch_bounds__(FT) void k_trsm_panel(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                   E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                                   const E* __restrict__ Dbuf) {
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  if (F.no <= k0) return;
  const int w = min(TB, F.no - k0);
  const int r0 = k0 + w + TB * blockIdx.y;
  if (r0 >= F.nf) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E As[TB * LDT];
  __shared__ E Bs[TB * LDT];
  const E* D = Dbuf + ((int64_t)t.doff[v] + k0 / TB) * (TB * TB);
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int i = idx % TB, k = idx / TB;        // row i of the tile, column k (coalesced in i)
    const int r = r0 + i;
    As[i * LDT + k] = (r < F.nf && k < w) ? F.L[(int64_t)(k0 + k) * F.nf + r] : E(0);
    const int kk = idx / TB, j = idx % TB;        // Bs[k][j] = D[j][k]
    Bs[kk * LDT + j] = D[j * TB + kk];
  }
  __syncthreads();
  acc_t<E> acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t<E>{0, 0, 0, 0};
  mma64<E>(As, Bs, w, acc, lane, wave, E(1));
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int r = r0 + acc_row<E>(lane, wave, ti, vv), c = acc_col(lane, wave, tj);
        if (r < F.nf && c < w) F.L[(int64_t)(k0 + c) * F.nf + r] = acc[ti][tj][vv];
      }
}

// Trailing update below the panel [k0, k0 + w): tiles (I, J), J <= I, of the
// front rows/columns from s0 = k0 + w, pair index in blockIdx.y.
template <class E>
__global__ __launch_bounds__(FT) void k_syrk_update(DevTree t, const int* __restrict__ level_nodes, int k0,
                                                    E* __restrict__ Lbuf, E* __restrict__ Ubuf) {
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E As[TB * LDT];
  __shared__ E Bs[TB * LDT];
  for (int idx = tid; idx < TB * TB; idx += FT) {
    const int i = idx % TB, k = idx / TB;
    const int ra = rI + i, rb = rJ + i;
    As[i * LDT + k] = (ra < F.nf && k < w) ? F.L[(int64_t)(k0 + k) * F.nf + ra] : E(0);
    Bs[k * LDT + i] = (rb < F.nf && k < w) ? F.L[(int64_t)(k0 + k) * F.nf + rb] : E(0);
  }
  __syncthreads();
  acc_t<E> acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int r = rI + acc_row<E>(lane, wave, ti, vv), c = rJ + acc_col(lane, wave, tj);
        acc[ti][tj][vv] = (r < F.nf && c < F.nf && r >= c) ? *F.at(r, c) : E(0);
      }
  mma64<E>(As, Bs, w, acc, lane, wave, E(-1));
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int r = rI + acc_row<E>(lane, wave, ti, vv), c = rJ + acc_col(lane, wave, tj);
        if (r < F.nf && c < F.nf && r >= c) *F.at(r, c) = acc[ti][tj][vv];
      }
}

// Rows [64 y, +64) of X with X L_oo = [I; L_bo]; X row r at T[r * no + ...].
template <class E>
__global__ __launch_bounds__(FT) void k_rtrsm(DevTree t, const int* __restrict__ level_nodes,
                                              E* __restrict__ Lbuf, E* __restrict__ Ubuf,
                                              E* __restrict__ Tbuf, const E* __restrict__ Dbuf) {
  const int v = level_nodes[blockIdx.x];
  const Front<E> F = front_of(t, v, Lbuf, Ubuf);
  const int nf = F.nf, no = F.no;
  const int r0 = TB * blockIdx.y;
  if (r0 >= nf || no == 0) return;
  E* T = Tbuf + t.loff[v];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ E As[TB * LDT];
  __shared__ E Bs[TB * LDT];
  const int npan = (no + TB - 1) / TB;
  const bool top = (r0 + TB <= no);            // every row of the block is an own row
  for (int P = npan - 1; P >= 0; --P) {
    const int c0 = P * TB, w = min(TB, no - c0);
    if (top && r0 + TB - 1 < c0) {               // X[r][c] = 0 for c > r < no
      for (int idx = tid; idx < TB * TB; idx += FT) {
        const int i = idx / TB, j = idx % TB;
        if (j < w) T[(int64_t)(r0 + i) * no + c0 + j] = E(0);
      }
      continue;
    }
    acc_t<E> acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int r = r0 + acc_row<E>(lane, wave, ti, vv), c = c0 + acc_col(lane, wave, tj);
          E val = E(0);
          if (r < nf && c < c0 + w) val = (r < no) ? (r == c ? E(1) : E(0)) : F.L[(int64_t)c * nf + r];
          acc[ti][tj][vv] = val;
        }
    // minus X[:, kb] L[kb, P] over solved block columns kb > P (X vanishes past the diagonal for top rows)
    const int kbmax = top ? min(npan - 1, (r0 + TB - 1) / TB) : npan - 1;
    for (int kb = P + 1; kb <= kbmax; ++kb) {
      const int cb = kb * TB, wb = min(TB, no - cb);
      __syncthreads();
      for (int idx = tid; idx < TB * TB; idx += FT) {
        const int k = idx % TB, i = idx / TB;      // As[i][k] = X[r0 + i][cb + k], coalesced in k
        As[i * LDT + k] = (r0 + i < nf && k < wb) ? T[(int64_t)(r0 + i) * no + cb + k] : E(0);
        const int j = idx / TB, kk = idx % TB;     // Bs[k][j] = L[cb + k][c0 + j], coalesced in k
        Bs[kk * LDT + j] = (kk < wb && j < w) ? F.L[(int64_t)(c0 + j) * nf + cb + kk] : E(0);
      }
      __syncthreads();
      mma64<E>(As, Bs, wb, acc, lane, wave, E(-1));
    }
    // X[:, P] = acc D_P
    __syncthreads();
    const E* D = Dbuf + ((int64_t)t.doff[v] + P) * (TB * TB);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv)
          As[acc_row<E>(lane, wave, ti, vv) * LDT + acc_col(lane, wave, tj)] = acc[ti][tj][vv];
    for (int idx = tid; idx < TB * TB; idx += FT) Bs[(idx / TB) * LDT + idx % TB] = D[idx];
    __syncthreads();
    acc_t<E> x[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) x[a][b] = acc_t<E>{0, 0, 0, 0};
    mma64<E>(As, Bs, w, x, lane, wave, E(1));
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int r = r0 + acc_row<E>(lane, wave, ti, vv), c = acc_col(lane, wave, tj);
          if (r < nf && c < w) T[(int64_t)r * no + c0 + c] = x[ti][tj][vv];
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
template <class E>
__global__ __launch_bounds__(FT) void k_pack(DevTree t, const int* __restrict__ level_nodes,
                                             const E* __restrict__ Tbuf, E* __restrict__ Lp, E* __restrict__ Tp) {
  constexpr int K = 16 / sizeof(E);
  const int v = level_nodes[blockIdx.x];
  const int nf = t.nf[v], no = t.no[v];
  const int nfp = (nf + K - 1) / K * K, nop = (no + K - 1) / K * K;
  const int ntr = (nfp + TB - 1) / TB;
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  const int r0 = tr * TB, c0 = tc * TB;
  if (r0 >= nfp || c0 >= nop) return;
  const E* T = Tbuf + t.loff[v];
  __shared__ E S[TB * LDT];
  for (int idx = threadIdx.x; idx < TB * TB; idx += FT) {
    const int i = idx / TB, c = idx % TB;         // row r0 + i, contiguous in c
    S[i * LDT + c] = (r0 + i < nf && c0 + c < no) ? T[(int64_t)(r0 + i) * no + c0 + c] : E(0);
  }
  __syncthreads();
  E* L = Lp + t.lpoff[v];
  for (int idx = threadIdx.x; idx < TB * TB; idx += FT) {
    const int gl = idx / (TB * K), rem = idx % (TB * K), r = rem / K, sl = rem % K;
    const int c = gl * K + sl;
    const int rr = r0 + r, g = (c0 + c) / K;
    if (rr < nf && c0 + c < nop && rr >= g * K) L[(lp_group(g, nf, K) + rr - g * K) * K + sl] = S[r * LDT + c];
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

template <class E>
void front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                  int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                  const double* C, E* L, E* U, E* T, E* D, E* Lp, E* Tp, const float* U32,
                  const double* U64, int64_t* status, hipStream_t st) {
  if (count <= 0) return;
  const int ncol = (max_nf + TB - 1) / TB;
  hipLaunchKernelGGL(k_front_assemble<E>, dim3(count, ncol), dim3(FT), (size_t)2 * max_nf * sizeof(int), st, s.n,
                     s.lo, s.hi, s.rowptr, t, level_nodes, s2, s1, K, M, C, L, U);
  if (max_child_nb > 0)
    for (int slot = 0; slot < max_kids; ++slot)
      hipLaunchKernelGGL(k_front_extend<E>, dim3(count, (max_child_nb + TB - 1) / TB), dim3(FT),
                         (size_t)max_child_nb * sizeof(int), st, t,
                         level_nodes, slot, L, U, U32, U64);
  for (int k0 = 0; k0 < max_no; k0 += TB) {
    hipLaunchKernelGGL(k_potrf_diag<E>, dim3(count), dim3(FT), 0, st, t, level_nodes, k0, L, U, D, status);
    // rows and trailing tiles below a block that is at least one column wide
    const int below = std::max(1, max_nf - k0 - 1);
    const int nrc = (below + TB - 1) / TB;
    hipLaunchKernelGGL(k_trsm_panel<E>, dim3(count, nrc), dim3(FT), 0, st, t, level_nodes, k0, L, U,
                       (const E*)D);
    hipLaunchKernelGGL(k_syrk_update<E>, dim3(count, nrc * (nrc + 1) / 2), dim3(FT), 0, st, t, level_nodes,
                       k0, L, U);
  }
  const int nrt = (max_nf + TB - 1) / TB;
  hipLaunchKernelGGL(k_rtrsm<E>, dim3(count, nrt), dim3(FT), 0, st, t, level_nodes, L, U, T, (const E*)D);
  const int nct = (max_no + 3 + TB - 1) / TB, nrp = (max_nf + 3 + TB - 1) / TB;
  hipLaunchKernelGGL(k_pack<E>, dim3(count, nrp * nct), dim3(FT), 0, st, t, level_nodes, (const E*)T, Lp, Tp);
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
