// B-spline tables and gather assembly of K, M, C (Sec. 3.1).
//
// The square uses the identity geometry and a tensor Gauss rule, so every
// 2-D element integral factorises into 1-D element integrals: for dofs
// a = (ax, ay), b = (bx, by) and element (ex, ey)
//   M_e[a,b] = m_ex[ax,bx] m_ey[ay,by],
//   K_e[a,b] = k_ex[ax,bx] m_ey[ay,by] + m_ex[ax,bx] k_ey[ay,by].
// Each CSR entry is produced by one thread that sums over the (at most
// (p+1)^2) elements shared by the two supports: a pure gather, no atomics, so
// the result is bitwise reproducible.
#include "kernels.hpp"

namespace riga {

constexpr int MAXP = 8;

// Nonzero degree-q B-splines at u inside knot span k (t[k] <= u < t[k+1]):
// the triangular Cox--de Boor scheme (eq. BasisFunBip), evaluated without
// forming the vanishing 0/0 terms.  N[r] is function k-q+r.
__device__ inline void basis_funs(int k, double u, int q, const int* t, double* N) {
  double left[MAXP + 1], right[MAXP + 1];
  N[0] = 1.0;
  for (int j = 1; j <= q; ++j) {
    left[j] = u - (double)t[k + 1 - j];
    right[j] = (double)t[k + j] - u;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      double tmp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

// Tables of element e of one 1-D space.
__device__ inline void element_tables(int e, int p, int ne, const int* __restrict__ knots,
                                      const int* __restrict__ first, const double* __restrict__ gx,
                                      const double* __restrict__ gw, double* __restrict__ tabM,
                                      double* __restrict__ tabK) {
  const int np = p + 1;
  const int k = first[e] + p;  // knot span of the element (knot indices are in element units)
  double m[(MAXP + 1) * (MAXP + 1)], kk[(MAXP + 1) * (MAXP + 1)];
  for (int a = 0; a < np * np; ++a) { m[a] = 0.0; kk[a] = 0.0; }
  for (int q = 0; q < np; ++q) {
    double u = (double)e + 0.5 * (gx[q] + 1.0);
    double w = 0.5 * gw[q];
    double N[MAXP + 1], Nm[MAXP + 1], D[MAXP + 1];
    basis_funs(k, u, p, knots, N);
    if (p > 1) basis_funs(k, u, p - 1, knots, Nm); else Nm[0] = 1.0;
    // dB_i/du = p (B_i^{p-1}/(t_{i+p}-t_i) - B_{i+1}^{p-1}/(t_{i+p+1}-t_{i+1})),
    // with Nm[s] the degree p-1 function k-p+1+s.
    for (int r = 0; r <= p; ++r) {
      int i = k - p + r;
      double d = 0.0;
      double d1 = (double)(knots[i + p] - knots[i]);
      double d2 = (double)(knots[i + p + 1] - knots[i + 1]);
      if (r >= 1 && d1 > 0.0) d += Nm[r - 1] / d1;
      if (r <= p - 1 && d2 > 0.0) d -= Nm[r] / d2;
      D[r] = (double)p * d;
    }
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        m[a * np + b] += w * N[a] * N[b];
        kk[a * np + b] += w * D[a] * D[b];
      }
  }
  // u = ne * x: dx = du / ne and d/dx = ne d/du
  const double h = 1.0 / (double)ne;
  for (int a = 0; a < np * np; ++a) {
    tabM[(int64_t)e * np * np + a] = m[a] * h;
    tabK[(int64_t)e * np * np + a] = kk[a] * (double)ne;
  }
}


__global__ void k_bspline_tables(int p, int ne, const int* __restrict__ knots, const int* __restrict__ first,
                                 const double* __restrict__ gx, const double* __restrict__ gw,
                                 double* __restrict__ tabM, double* __restrict__ tabK) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) element_tables(e, p, ne, knots, first, gx, gw, tabM, tabK);
}

// Every problem of a forest: problem blockIdx.y, its tables at tabM/tabK +
// taboff[problem], its Gauss rule at gx[problem], gw[problem].
__global__ void k_bspline_tables_b(const DevSpace* __restrict__ spaces, const int64_t* __restrict__ taboff,
                                   const double* const* __restrict__ gx, const double* const* __restrict__ gw,
                                   double* __restrict__ tabM, double* __restrict__ tabK) {
  const int q = blockIdx.y;
  const DevSpace sp = spaces[q];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < sp.ne) element_tables(e, sp.p, sp.ne, sp.knots, sp.first, gx[q], gw[q], tabM + taboff[q], tabK + taboff[q]);
}

void launch_bspline_tables(const DevSpace& s, const double* gx, const double* gw,
                           double* tabM, double* tabK, hipStream_t st) {
  int threads = 64;
  int blocks = (s.ne + threads - 1) / threads;
  hipLaunchKernelGGL(k_bspline_tables, dim3(blocks), dim3(threads), 0, st,
                     s.p, s.ne, s.knots, s.first, gx, gw, tabM, tabK);
}

constexpr int ASM_ROWS = 64;
constexpr int ASM_THREADS = 256;
constexpr int ASM_MAXROWS = 256;   // rows of one block at most (forest row blocks)

// Entries of rows [r0, r0 + nrows) of one space (row indices local to the
// space, rowptr its row pointers into the value arrays); rp: nrows + 1 words
// of shared memory.
__device__ inline void assemble_rows(const DevSpace& s, int64_t r0, int nrows, const double* __restrict__ tabM,
                                     const double* __restrict__ tabK, double alpha, double beta,
                                     const double* __restrict__ c_elem, double* __restrict__ Ko,
                                     double* __restrict__ Mo, double* __restrict__ Co, int64_t* rp) {
  const int p = s.p, ne = s.ne, n = s.n;
  const int *sup0 = s.sup0, *sup1 = s.sup1, *lo = s.lo, *hi = s.hi, *first = s.first;
  for (int t = threadIdx.x; t <= nrows; t += blockDim.x) rp[t] = s.rowptr[r0 + t];
  __syncthreads();
  const int np = p + 1;
  const int64_t kbeg = rp[0], kend = rp[nrows];
  for (int64_t k = kbeg + threadIdx.x; k < kend; k += blockDim.x) {
    // row of entry k: last row whose start is <= k
    int a = 0, b = nrows;  // invariant rp[a] <= k < rp[b]
    while (b - a > 1) {
      int c = (a + b) >> 1;
      if (rp[c] <= k) a = c; else b = c;
    }
    const int64_t r = r0 + a;
    const int i = (int)(r % n), j = (int)(r / n);
    const int o = (int)(k - rp[a]);
    const int wx = hi[i] - lo[i] + 1;
    const int jj = lo[j] + o / wx, ii = lo[i] + o % wx;
    // x factor: elements shared by the supports of functions i and ii
    double mx[MAXP + 1], my[MAXP + 1];
    double sx = 0.0, kx = 0.0, sy = 0.0, ky = 0.0;
    const int ex0 = max(sup0[i], sup0[ii]), ex1 = min(sup1[i], sup1[ii]);
    for (int ex = ex0; ex < ex1; ++ex) {
      int la = i + 1 - first[ex], lb = ii + 1 - first[ex];
      int64_t idx = (int64_t)ex * np * np + la * np + lb;
      mx[ex - ex0] = tabM[idx];
      sx += tabM[idx];
      kx += tabK[idx];
    }
    const int ey0 = max(sup0[j], sup0[jj]), ey1 = min(sup1[j], sup1[jj]);
    for (int ey = ey0; ey < ey1; ++ey) {
      int la = j + 1 - first[ey], lb = jj + 1 - first[ey];
      int64_t idx = (int64_t)ey * np * np + la * np + lb;
      my[ey - ey0] = tabM[idx];
      sy += tabM[idx];
      ky += tabK[idx];
    }
    const double mval = sx * sy;
    const double kval = kx * sy + sx * ky;
    double cval = alpha * mval + beta * kval;
    if (c_elem) {
      double acc = 0.0;
      for (int ey = ey0; ey < ey1; ++ey) {
        double rowacc = 0.0;
        for (int ex = ex0; ex < ex1; ++ex) rowacc += c_elem[(int64_t)ey * ne + ex] * mx[ex - ex0];
        acc += rowacc * my[ey - ey0];
      }
      cval += acc;
    }
    Ko[k] = kval;
    Mo[k] = mval;
    Co[k] = cval;
  }
}

__global__ __launch_bounds__(ASM_THREADS) void k_assemble(DevSpace s, int64_t ndof, const double* __restrict__ tabM,
                                                          const double* __restrict__ tabK, double alpha, double beta,
                                                          const double* __restrict__ c_elem, double* __restrict__ Ko,
                                                          double* __restrict__ Mo, double* __restrict__ Co) {
  __shared__ int64_t rp[ASM_ROWS + 1];
  const int64_t r0 = (int64_t)blockIdx.x * ASM_ROWS;
  assemble_rows(s, r0, (int)min((int64_t)ASM_ROWS, ndof - r0), tabM, tabK, alpha, beta, c_elem, Ko, Mo, Co, rp);
}

// Every problem of a forest, one block per row block rb[b] = {problem, first
// row, end row} (forest rows; the problem's rows start at dofbase).
__global__ __launch_bounds__(ASM_THREADS) void k_assemble_b(const int4* __restrict__ rb,
                                                            const DevSpace* __restrict__ spaces,
                                                            const int64_t* __restrict__ dofbase,
                                                            const int64_t* __restrict__ taboff,
                                                            const double* __restrict__ tabM,
                                                            const double* __restrict__ tabK,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta,
                                                            const double* const* __restrict__ c_elem,
                                                            double* __restrict__ Ko, double* __restrict__ Mo,
                                                            double* __restrict__ Co) {
  __shared__ int64_t rp[ASM_MAXROWS + 1];
  const int4 b = rb[blockIdx.x];
  const int q = b.x;
  const DevSpace sp = spaces[q];
  assemble_rows(sp, b.y - dofbase[q], b.z - b.y, tabM + taboff[q], tabK + taboff[q], alpha[q], beta[q], c_elem[q],
                Ko, Mo, Co, rp);
}

void launch_assemble_b(const int4* rb, int nrb, const DevSpace* spaces, const int64_t* dofbase,
                       const int64_t* taboff, const double* const* gx, const double* const* gw, int n, int max_ne,
                       double* tabM, double* tabK, const double* alpha, const double* beta,
                       const double* const* c_elem, double* K, double* M, double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_bspline_tables_b, dim3((max_ne + 63) / 64, n), dim3(64), 0, st, spaces, taboff, gx, gw, tabM,
                     tabK);
  hipLaunchKernelGGL(k_assemble_b, dim3(nrb), dim3(ASM_THREADS), 0, st, rb, spaces, dofbase, taboff, tabM, tabK,
                     alpha, beta, c_elem, K, M, C);
}

// Banded 1-D mass and stiffness matrices of one space: entry (i, ii), ii in
// lo[i] .. hi[i], is the sum over the shared elements that assemble_rows forms
// for its x factor (same terms, same order), stored at i (2p + 1) + ii - i + p;
// every other slot of the band is zero.  M = M1 (x) M1 and
// K = K1 (x) M1 + M1 (x) K1 on the tensor grid.
__device__ inline void band_entry(const DevSpace& s, int i, int o, const double* __restrict__ tabM,
                                  const double* __restrict__ tabK, double* __restrict__ M1, double* __restrict__ K1) {
  const int p = s.p, np = p + 1, w = 2 * p + 1;
  const int ii = i - p + o;
  double sx = 0.0, kx = 0.0;
  if (ii >= s.lo[i] && ii <= s.hi[i]) {
    const int ex0 = max(s.sup0[i], s.sup0[ii]), ex1 = min(s.sup1[i], s.sup1[ii]);
    for (int ex = ex0; ex < ex1; ++ex) {
      const int la = i + 1 - s.first[ex], lb = ii + 1 - s.first[ex];
      const int64_t idx = (int64_t)ex * np * np + la * np + lb;
      sx += tabM[idx];
      kx += tabK[idx];
    }
  }
  M1[(int64_t)i * w + o] = sx;
  K1[(int64_t)i * w + o] = kx;
}

__global__ void k_band_1d(DevSpace s, const double* __restrict__ tabM, const double* __restrict__ tabK,
                          double* __restrict__ M1, double* __restrict__ K1) {
  const int w = 2 * s.p + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < s.n * w) band_entry(s, t / w, t % w, tabM, tabK, M1, K1);
}

void launch_band_1d(const DevSpace& s, const double* tabM, const double* tabK, double* M1, double* K1,
                    hipStream_t st) {
  const int total = s.n * (2 * s.p + 1);
  hipLaunchKernelGGL(k_band_1d, dim3((total + 255) / 256), dim3(256), 0, st, s, tabM, tabK, M1, K1);
}

__global__ void k_band_1d_b(const DevSpace* __restrict__ spaces, const int64_t* __restrict__ taboff,
                            const double* __restrict__ tabM, const double* __restrict__ tabK,
                            const int64_t* __restrict__ bandoff, double* __restrict__ M1, double* __restrict__ K1) {
  const int q = blockIdx.y;
  const DevSpace sp = spaces[q];
  const int w = 2 * sp.p + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < sp.n * w)
    band_entry(sp, t / w, t % w, tabM + taboff[q], tabK + taboff[q], M1 + bandoff[q], K1 + bandoff[q]);
}

void launch_band_1d_b(const DevSpace* spaces, int n, int max_w, const int64_t* taboff, const double* tabM,
                      const double* tabK, const int64_t* bandoff, double* M1, double* K1, hipStream_t st) {
  hipLaunchKernelGGL(k_band_1d_b, dim3((max_w + 255) / 256, n), dim3(256), 0, st, spaces, taboff, tabM, tabK, bandoff,
                     M1, K1);
}

void launch_assemble(const DevSpace& s, const double* tabM, const double* tabK,
                     double alpha, double beta, const double* c_elem,
                     double* K, double* M, double* C, int64_t ndof, hipStream_t st) {
  int64_t blocks = (ndof + ASM_ROWS - 1) / ASM_ROWS;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(ASM_THREADS), 0, st, s, ndof, tabM, tabK, alpha, beta,
                     c_elem, K, M, C);
}
}  // namespace riga
