// B-spline tables and gather assembly of K, M, C (Sec. 3.1).
//
// The square uses the identity geometry and a tensor Gauss rule, so every
// 2-D element integral factorises into 1-D element integrals: for dofs
// a = (ax, ay), b = (bx, by) and element (ex, ey)
//   M_e[a,b] = m_ex[ax,bx] m_ey[ay,by],
//   K_e[a,b] = k_ex[ax,bx] m_ey[ay,by] + m_ex[ax,bx] k_ey[ay,by].
// The 1-D factors are assembled first as bands (k_band_1d: m_x and k_x summed
// over the elements two supports share), and every CSR row of M, K, C is then
// written by one wave from the two band rows of its dof, lane = stored entry:
//   M = M1[i][ii] M1[j][jj],  K = K1[i][ii] M1[j][jj] + M1[i][ii] K1[j][jj],
// consecutive lanes writing consecutive entries.  A per-element damping field
// adds sum_{ey, ex} c[ey][ex] m_ex[i, ii] m_ey[j, jj], formed per row through
// the table T[ey][ii] = sum_ex c[ey][ex] m_ex[i, ii] (in LDS).  A pure gather,
// no atomics, so the result is bitwise reproducible.
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
// tabS (may be null): the element integrals of B_a dB_b/dx (the skew form of
// a gyroscopic damping).
__device__ inline void element_tables(int e, int p, int ne, const int* __restrict__ knots,
                                      const int* __restrict__ first, const double* __restrict__ gx,
                                      const double* __restrict__ gw, double* __restrict__ tabM,
                                      double* __restrict__ tabK, double* __restrict__ tabS = nullptr) {
  const int np = p + 1;
  const int k = first[e] + p;  // knot span of the element (knot indices are in element units)
  double m[(MAXP + 1) * (MAXP + 1)], kk[(MAXP + 1) * (MAXP + 1)], sk[(MAXP + 1) * (MAXP + 1)];
  for (int a = 0; a < np * np; ++a) { m[a] = 0.0; kk[a] = 0.0; sk[a] = 0.0; }
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
        sk[a * np + b] += w * N[a] * D[b];
      }
  }
  // u = ne * x: dx = du / ne and d/dx = ne d/du (B dB/dx dx = B dB/du du)
  const double h = 1.0 / (double)ne;
  for (int a = 0; a < np * np; ++a) {
    tabM[(int64_t)e * np * np + a] = m[a] * h;
    tabK[(int64_t)e * np * np + a] = kk[a] * (double)ne;
    if (tabS != nullptr) tabS[(int64_t)e * np * np + a] = sk[a];
  }
}


__global__ void k_bspline_tables(int p, int ne, const int* __restrict__ knots, const int* __restrict__ first,
                                 const double* __restrict__ gx, const double* __restrict__ gw,
                                 double* __restrict__ tabM, double* __restrict__ tabK, double* __restrict__ tabS) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) element_tables(e, p, ne, knots, first, gx, gw, tabM, tabK, tabS);
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
                           double* tabM, double* tabK, double* tabS, hipStream_t st) {
  int threads = 64;
  int blocks = (s.ne + threads - 1) / threads;
  hipLaunchKernelGGL(k_bspline_tables, dim3(blocks), dim3(threads), 0, st,
                     s.p, s.ne, s.knots, s.first, gx, gw, tabM, tabK, tabS);
}

constexpr int ASM_THREADS = 256;
constexpr int ASM_WAVES = ASM_THREADS / 64;
constexpr int ASM_ROWS_PER_WAVE = 4;
constexpr int ASM_TMAX = (MAXP + 1) * (2 * MAXP + 1);   // T[ey][ii] entries per row

// Row r (local to the space, uniform in the wave) of K, M, C from the bands
// M1, K1 (row i at i (2p + 1), column ii at + ii - i + p); T: ASM_TMAX doubles
// of this wave's shared memory.
// With S1 (the band of s_ij = int B_i B_j', null otherwise) C gains the skew
// gyroscopic part g = gx S1[i][ii] M1[j][jj] + gy M1[i][ii] S1[j][jj] and Cto
// receives the transpose's values on the same pattern (C^T = sym - g).
__device__ inline void assemble_row(const DevSpace& s, int64_t r, const double* __restrict__ tabM,
                                    const double* __restrict__ M1, const double* __restrict__ K1, double alpha,
                                    double beta, const double* __restrict__ c_elem, double* __restrict__ Ko,
                                    double* __restrict__ Mo, double* __restrict__ Co, double* T, int lane,
                                    const double* __restrict__ S1 = nullptr, double gxs = 0.0, double gys = 0.0,
                                    double* __restrict__ Cto = nullptr) {
  const int p = s.p, n = s.n, ne = s.ne, w = 2 * p + 1, np = p + 1;
  const int i = (int)(r % n), j = (int)(r / n);
  const int lox = s.lo[i], wx = s.hi[i] - lox + 1, loy = s.lo[j];
  const int64_t k0 = s.rowptr[r];
  const int len = (int)(s.rowptr[r + 1] - k0);
  const double* mxr = M1 + (int64_t)i * w - i + p;   // mxr[ii] = M1[i][ii]
  const double* kxr = K1 + (int64_t)i * w - i + p;
  const double* myr = M1 + (int64_t)j * w - j + p;
  const double* kyr = K1 + (int64_t)j * w - j + p;
  const double* sxr = S1 ? S1 + (int64_t)i * w - i + p : nullptr;
  const double* syr = S1 ? S1 + (int64_t)j * w - j + p : nullptr;
  const int sy0 = s.sup0[j], sy1 = s.sup1[j];
  if (c_elem != nullptr) {
    // T[ey - sy0][ii - lox] over the elements ey of j's support and the
    // coupled functions ii of i
    const int nt = (sy1 - sy0) * wx;
    for (int t = lane; t < nt; t += 64) {
      const int ey = sy0 + t / wx, ii = lox + t % wx;
      const int ex0 = max(s.sup0[i], s.sup0[ii]), ex1 = min(s.sup1[i], s.sup1[ii]);
      double acc = 0.0;
      for (int ex = ex0; ex < ex1; ++ex) {
        const int fx = s.first[ex];
        acc += c_elem[(int64_t)ey * ne + ex] * tabM[((int64_t)ex * np + i + 1 - fx) * np + ii + 1 - fx];
      }
      T[t] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  for (int o = lane; o < len; o += 64) {
    const int jj = loy + o / wx, ii = lox + o % wx;
    const double mx = mxr[ii], kx = kxr[ii], my = myr[jj], ky = kyr[jj];
    const double mval = mx * my;
    const double kval = kx * my + mx * ky;
    double cval = alpha * mval + beta * kval;
    if (c_elem != nullptr) {
      const int ey0 = max(sy0, s.sup0[jj]), ey1 = min(sy1, s.sup1[jj]);
      double acc = 0.0;
      for (int ey = ey0; ey < ey1; ++ey) {
        const int fy = s.first[ey];
        acc += tabM[((int64_t)ey * np + j + 1 - fy) * np + jj + 1 - fy] * T[(ey - sy0) * wx + ii - lox];
      }
      cval += acc;
    }
    Ko[k0 + o] = kval;
    Mo[k0 + o] = mval;
    if (S1 != nullptr) {
      const double g = gxs * sxr[ii] * my + gys * mx * syr[jj];
      Co[k0 + o] = cval + g;
      Cto[k0 + o] = cval - g;
    } else {
      Co[k0 + o] = cval;
    }
  }
}

__global__ __launch_bounds__(ASM_THREADS) void k_assemble(DevSpace s, int64_t ndof, const double* __restrict__ tabM,
                                                          const double* __restrict__ M1, const double* __restrict__ K1,
                                                          double alpha, double beta,
                                                          const double* __restrict__ c_elem, double* __restrict__ Ko,
                                                          double* __restrict__ Mo, double* __restrict__ Co,
                                                          const double* __restrict__ S1, double gxs, double gys,
                                                          double* __restrict__ Cto) {
  __shared__ double T[ASM_WAVES][ASM_TMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * ASM_WAVES + wave) * ASM_ROWS_PER_WAVE;
  for (int q = 0; q < ASM_ROWS_PER_WAVE; ++q) {
    const int64_t r = r0 + q;
    if (r >= ndof) break;
    assemble_row(s, r, tabM, M1, K1, alpha, beta, c_elem, Ko, Mo, Co, T[wave], lane, S1, gxs, gys, Cto);
  }
}

// Every problem of a forest, one block per row block rb[b] = {problem, first
// row, end row} (forest rows; the problem's rows start at dofbase), the waves
// taking its rows in turn; bands at M1 / K1 + bandoff[q].
__global__ __launch_bounds__(ASM_THREADS) void k_assemble_b(const int4* __restrict__ rb,
                                                            const DevSpace* __restrict__ spaces,
                                                            const int64_t* __restrict__ dofbase,
                                                            const int64_t* __restrict__ taboff,
                                                            const double* __restrict__ tabM,
                                                            const int64_t* __restrict__ bandoff,
                                                            const double* __restrict__ M1,
                                                            const double* __restrict__ K1,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta,
                                                            const double* const* __restrict__ c_elem,
                                                            double* __restrict__ Ko, double* __restrict__ Mo,
                                                            double* __restrict__ Co) {
  __shared__ double T[ASM_WAVES][ASM_TMAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int4 b = rb[blockIdx.x];
  const int q = b.x;
  const DevSpace sp = spaces[q];
  const int64_t base = dofbase[q];
  for (int64_t row = b.y + wave; row < b.z; row += ASM_WAVES)
    assemble_row(sp, row - base, tabM + taboff[q], M1 + bandoff[q], K1 + bandoff[q], alpha[q], beta[q], c_elem[q], Ko,
                 Mo, Co, T[wave], lane);
}

void launch_assemble_b(const int4* rb, int nrb, const DevSpace* spaces, const int64_t* dofbase,
                       const int64_t* taboff, const double* const* gx, const double* const* gw, int n, int max_ne,
                       double* tabM, double* tabK, int max_w, const int64_t* bandoff, double* M1, double* K1,
                       const double* alpha, const double* beta, const double* const* c_elem, double* K, double* M,
                       double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_bspline_tables_b, dim3((max_ne + 63) / 64, n), dim3(64), 0, st, spaces, taboff, gx, gw, tabM,
                     tabK);
  launch_band_1d_b(spaces, n, max_w, taboff, tabM, tabK, bandoff, M1, K1, st);
  hipLaunchKernelGGL(k_assemble_b, dim3(nrb), dim3(ASM_THREADS), 0, st, rb, spaces, dofbase, taboff, tabM, bandoff,
                     M1, K1, alpha, beta, c_elem, K, M, C);
}

// Banded 1-D mass and stiffness matrices of one space: entry (i, ii), ii in
// lo[i] .. hi[i], is the sum of the element blocks over the elements the two
// supports share, stored at i (2p + 1) + ii - i + p;
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

// Band of the 1-D skew matrix s_ij = int B_i B_j' (same layout as M1, K1).
__global__ void k_band_skew(DevSpace s, const double* __restrict__ tabS, double* __restrict__ S1) {
  const int p = s.p, np = p + 1, w = 2 * p + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s.n * w) return;
  const int i = t / w, ii = i - p + t % w;
  double v = 0.0;
  if (ii >= s.lo[i] && ii <= s.hi[i]) {
    const int ex0 = max(s.sup0[i], s.sup0[ii]), ex1 = min(s.sup1[i], s.sup1[ii]);
    for (int ex = ex0; ex < ex1; ++ex) {
      const int la = i + 1 - s.first[ex], lb = ii + 1 - s.first[ex];
      v += tabS[(int64_t)ex * np * np + la * np + lb];
    }
  }
  S1[t] = v;
}

void launch_band_skew(const DevSpace& s, const double* tabS, double* S1, hipStream_t st) {
  const int total = s.n * (2 * s.p + 1);
  hipLaunchKernelGGL(k_band_skew, dim3((total + 255) / 256), dim3(256), 0, st, s, tabS, S1);
}

void launch_assemble(const DevSpace& s, const double* tabM, const double* M1, const double* K1,
                     double alpha, double beta, const double* c_elem,
                     double* K, double* M, double* C, int64_t ndof, hipStream_t st,
                     const double* S1, double gx, double gy, double* Ct) {
  const int64_t rows = (int64_t)ASM_WAVES * ASM_ROWS_PER_WAVE;
  const int64_t blocks = (ndof + rows - 1) / rows;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(ASM_THREADS), 0, st, s, ndof, tabM, M1, K1, alpha, beta,
                     c_elem, K, M, C, S1, gx, gy, Ct);
}

// ---------------------------------------------------------------------------
// H(curl) space S^{p-1,p} x S^{p,p-1} (Sec. 3.2, eq. HcurlBasis): component 0
// dofs (i, j) = A_i(x) B_j(y) first, component 1 dofs B_i(x) A_j(y) from base1
// on (x fastest within a component), with A the degree-(p-1) and B the
// degree-p 1-D space.  With rot u = d u_2/dx - d u_1/dy,
//   K00 = MA[i][ii] KB[j][jj],   K11 = KB[i][ii] MA[j][jj],
//   K01 = -D[i][ii] D[jj][j],    K10 = -D[ii][i] D[j][jj],
//   M00 = MA[i][ii] MB[j][jj],   M11 = MB[i][ii] MA[j][jj],   M01 = M10 = 0,
// with MA, MB, KB, D the dense 1-D matrices (hcurl_1d on the host); C =
// alpha M + beta K.  One wave per row, lanes over its stored entries
// (explicit column indices).
__global__ __launch_bounds__(ASM_THREADS) void k_assemble_hcurl(int na, int nb, int64_t base1, int64_t ndof,
                                                                const int64_t* __restrict__ rowptr,
                                                                const int* __restrict__ col,
                                                                const double* __restrict__ MA,
                                                                const double* __restrict__ MB,
                                                                const double* __restrict__ KB,
                                                                const double* __restrict__ D, double alpha,
                                                                double beta, double* __restrict__ Ko,
                                                                double* __restrict__ Mo, double* __restrict__ Co) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * ASM_WAVES + wave) * ASM_ROWS_PER_WAVE;
  for (int qr = 0; qr < ASM_ROWS_PER_WAVE; ++qr) {
    const int64_t r = r0 + qr;
    if (r >= ndof) break;
    const int c = r >= base1 ? 1 : 0;
    const int64_t rr = r - (c ? base1 : 0);
    const int nx = c ? nb : na;
    const int i = (int)(rr % nx), j = (int)(rr / nx);
    const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
    for (int64_t k = k0 + lane; k < k1; k += 64) {
      const int64_t cc = col[k];
      const int b = cc >= base1 ? 1 : 0;
      const int64_t cr = cc - (b ? base1 : 0);
      const int mx = b ? nb : na;
      const int ii = (int)(cr % mx), jj = (int)(cr / mx);
      double kv, mv;
      if (c == 0 && b == 0) {
        kv = MA[(int64_t)i * na + ii] * KB[(int64_t)j * nb + jj];
        mv = MA[(int64_t)i * na + ii] * MB[(int64_t)j * nb + jj];
      } else if (c == 1 && b == 1) {
        kv = KB[(int64_t)i * nb + ii] * MA[(int64_t)j * na + jj];
        mv = MB[(int64_t)i * nb + ii] * MA[(int64_t)j * na + jj];
      } else if (c == 0) {
        kv = -D[(int64_t)i * nb + ii] * D[(int64_t)jj * nb + j];
        mv = 0.0;
      } else {
        kv = -D[(int64_t)ii * nb + i] * D[(int64_t)j * nb + jj];
        mv = 0.0;
      }
      Ko[k] = kv;
      Mo[k] = mv;
      Co[k] = alpha * mv + beta * kv;
    }
  }
}

// Rows of the divergence-conforming space S^{p,p-1} x S^{p-1,p} (eq.
// HdivBasis) and the vibroacoustic forms of Sec. 2.2 (rho = c = 1): component 0
// is Bx_i(x) A_j(y), component 1 is A_i(x) By_j(y), div u = d/dx of component
// 0 plus d/dy of component 1, so on the identity geometry
//   K00 = KBx (x) MA,  K11 = MA (x) KBy,
//   K01 = Dx[ii][i] Dy[j][jj],  K10 = Dx[i][ii] Dy[jj][j]   (D = int A B'),
//   M00 = MBx (x) MA,  M11 = MA (x) MBy,  M01 = M10 = 0,
// plus the absorbing walls' G = int (u.n)(v.n): on an x wall the end function
// of Bx (1 there) times MA in y, on a y wall MA in x times the end function of
// By; K = Kdiv + alpha G, M, C = beta G.  One wave per row (see k_assemble).
__global__ __launch_bounds__(ASM_THREADS) void k_assemble_hdiv(
    int na, int nbx, int nby, int64_t base1, int64_t ndof, const int64_t* __restrict__ rowptr,
    const int* __restrict__ col, const double* __restrict__ MA, const double* __restrict__ MBx,
    const double* __restrict__ KBx, const double* __restrict__ Dx, const double* __restrict__ MBy,
    const double* __restrict__ KBy, const double* __restrict__ Dy, int wl, int wr, int wb, int wt, double alpha,
    double beta, double* __restrict__ Ko, double* __restrict__ Mo, double* __restrict__ Co) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * ASM_WAVES + wave) * ASM_ROWS_PER_WAVE;
  for (int qr = 0; qr < ASM_ROWS_PER_WAVE; ++qr) {
    const int64_t r = r0 + qr;
    if (r >= ndof) break;
    const int c = r >= base1 ? 1 : 0;
    const int64_t rr = r - (c ? base1 : 0);
    const int nx = c ? na : nbx;
    const int i = (int)(rr % nx), j = (int)(rr / nx);
    const int64_t k0 = rowptr[r], k1 = rowptr[r + 1];
    for (int64_t k = k0 + lane; k < k1; k += 64) {
      const int64_t cc = col[k];
      const int b = cc >= base1 ? 1 : 0;
      const int64_t cr = cc - (b ? base1 : 0);
      const int mx = b ? na : nbx;
      const int ii = (int)(cr % mx), jj = (int)(cr / mx);
      double kv, mv, gv = 0.0;
      if (c == 0 && b == 0) {
        kv = KBx[(int64_t)i * nbx + ii] * MA[(int64_t)j * na + jj];
        mv = MBx[(int64_t)i * nbx + ii] * MA[(int64_t)j * na + jj];
        // x walls: the first (left) or last (right) kept function of Bx
        const bool lw = wl && i == 0 && ii == 0, rw = wr && i == nbx - 1 && ii == nbx - 1;
        if (lw || rw) gv = MA[(int64_t)j * na + jj] * ((lw ? 1.0 : 0.0) + (rw ? 1.0 : 0.0));
      } else if (c == 1 && b == 1) {
        kv = MA[(int64_t)i * na + ii] * KBy[(int64_t)j * nby + jj];
        mv = MA[(int64_t)i * na + ii] * MBy[(int64_t)j * nby + jj];
        const bool bw = wb && j == 0 && jj == 0, tw = wt && j == nby - 1 && jj == nby - 1;
        if (bw || tw) gv = MA[(int64_t)i * na + ii] * ((bw ? 1.0 : 0.0) + (tw ? 1.0 : 0.0));
      } else if (c == 0) {
        kv = Dx[(int64_t)ii * nbx + i] * Dy[(int64_t)j * nby + jj];
        mv = 0.0;
      } else {
        kv = Dx[(int64_t)i * nbx + ii] * Dy[(int64_t)jj * nby + j];
        mv = 0.0;
      }
      Ko[k] = kv + alpha * gv;
      Mo[k] = mv;
      Co[k] = beta * gv;
    }
  }
}

void launch_assemble_hdiv(int na, int nbx, int nby, int64_t base1, int64_t ndof, const int64_t* rowptr,
                          const int* col, const double* MA, const double* MBx, const double* KBx, const double* Dx,
                          const double* MBy, const double* KBy, const double* Dy, int walls, double alpha,
                          double beta, double* K, double* M, double* C, hipStream_t st) {
  const int64_t rows = (int64_t)ASM_WAVES * ASM_ROWS_PER_WAVE;
  const int64_t blocks = (ndof + rows - 1) / rows;
  hipLaunchKernelGGL(k_assemble_hdiv, dim3((unsigned)blocks), dim3(ASM_THREADS), 0, st, na, nbx, nby, base1, ndof,
                     rowptr, col, MA, MBx, KBx, Dx, MBy, KBy, Dy, walls & 1, (walls >> 1) & 1, (walls >> 2) & 1,
                     (walls >> 3) & 1, alpha, beta, K, M, C);
}

void launch_assemble_hcurl(int na, int nb, int64_t base1, int64_t ndof, const int64_t* rowptr, const int* col,
                           const double* MA, const double* MB, const double* KB, const double* D, double alpha,
                           double beta, double* K, double* M, double* C, hipStream_t st) {
  const int64_t rows = (int64_t)ASM_WAVES * ASM_ROWS_PER_WAVE;
  const int64_t blocks = (ndof + rows - 1) / rows;
  hipLaunchKernelGGL(k_assemble_hcurl, dim3((unsigned)blocks), dim3(ASM_THREADS), 0, st, na, nb, base1, ndof, rowptr,
                     col, MA, MB, KB, D, alpha, beta, K, M, C);
}

}  // namespace riga
