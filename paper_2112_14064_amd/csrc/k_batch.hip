// Batched form: the Krylov building blocks for a forest of independent QEPs
// of different sizes, run in lockstep (one launch per operation for all of
// them).  Every problem owns a contiguous range of rows of the forest vectors
// (dofbase); per-problem state lives on the device (current column k, live
// flag, small matrices at fixed strides), so one captured block step replays
// unchanged for every step of every problem.  Row-parallel kernels take a
// table of row blocks that never straddle two problems:
//   rb[blk] = {problem, first row, end row, 0}.
#include "kernels.hpp"
#include "krylov_dev.hpp"

#include <algorithm>

namespace riga {

constexpr int BT = 256;   // threads per block of the row-parallel kernels

// A = sigma_p M + C on every problem's rows (nonzero ranges nzbase[p] .. nzbase[p+1]).
__global__ __launch_bounds__(BT) void k_combine_b(int n, const int64_t* __restrict__ nzbase,
                                                  const double* __restrict__ sig, const double* __restrict__ M,
                                                  const double* __restrict__ C, double* __restrict__ A) {
  const int64_t nnz = nzbase[n];
  for (int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * BT) {
    int a = 0, b = n;   // nzbase[a] <= k < nzbase[b]
    while (b - a > 1) {
      const int c = (a + b) >> 1;
      if (nzbase[c] <= k) a = c; else b = c;
    }
    A[k] = sig[a] * M[k] + C[k];
  }
}

void launch_combine_b(int n, const int64_t* nzbase, int64_t nnz, const double* sig, const double* M, const double* C,
                      double* A, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((nnz + BT - 1) / BT, 8192);
  hipLaunchKernelGGL(k_combine_b, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(BT), 0, st, n, nzbase, sig, M, C,
                     A);
}

// Xu[:, q] = Vu[:, k + q], Xw[:, q] = Wl[:, k + q] with k the problem's current column.
__global__ __launch_bounds__(BT) void k_gather_b(const int4* __restrict__ rb, const int* __restrict__ kcur,
                                                 const unsigned char* __restrict__ live, int nq,
                                                 const double* __restrict__ Vu, const double* __restrict__ Wl,
                                                 int64_t ld, double* __restrict__ Xu, double* __restrict__ Xw) {
  const int4 b = rb[blockIdx.x];
  if (live && !live[b.x]) return;
  const int64_t r = b.y + threadIdx.x;
  if (r >= b.z) return;
  const int k = kcur[b.x];
  for (int q = 0; q < nq; ++q) {
    Xu[r + q * ld] = Vu[r + (int64_t)(k + q) * ld];
    Xw[r + q * ld] = Wl[r + (int64_t)(k + q) * ld];
  }
}

void launch_gather_b(const BatchDev& B, int nq, const double* Vu, const double* Wl, double* Xu, double* Xw,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gather_b, dim3(B.nrb), dim3(BT), 0, st, B.rb, B.kcur, B.live, nq, Vu, Wl, B.ntot, Xu, Xw);
}

// Partial multi-dots per dot block (rows of one problem):
// partial[blk * pstride + c * NQ + q] = sum_rows Au[:, c] Xu[:, q] + Al[:, c] Xl[:, q],
// c < nc = kcur[p] + nc_add (or nc_fixed without kcur).
template <int NQ>
__global__ __launch_bounds__(BT) void k_dots_b(const int4* __restrict__ db, const int* __restrict__ kcur,
                                               int nc_add, int nc_fixed, const unsigned char* __restrict__ live,
                                               const double* __restrict__ Au, const double* __restrict__ Al,
                                               int64_t lda, const double* __restrict__ Xu,
                                               const double* __restrict__ Xl, int64_t ldx,
                                               double* __restrict__ partial, int pstride) {
  const int4 b = db[blockIdx.x];
  if (live && !live[b.x]) return;
  const int nc = kcur ? kcur[b.x] + nc_add : nc_fixed;
  const int64_t i0 = b.y, i1 = b.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* out = partial + (int64_t)blockIdx.x * pstride;
  dots_body<NQ, BT / 64>(i0, i1, nc, Au, Al, lda, Xu, Xl, ldx, NQ, nullptr, nullptr, lane, wave,
                         [&](int c, int q, double v) { out[c * NQ + q] = v; });
}

// out[p * ostride + idx] = sum over the problem's dot blocks of the partials
// (fixed order: deterministic), one workgroup per problem.
__global__ __launch_bounds__(BT) void k_dots_final_b(const int* __restrict__ dboff, const int* __restrict__ kcur,
                                                     int nc_add, int nc_fixed, const unsigned char* __restrict__ live,
                                                     int nq, const double* __restrict__ partial, int pstride,
                                                     double* __restrict__ out, int ostride) {
  const int p = blockIdx.x;
  if (live && !live[p]) return;
  const int nout = (kcur ? kcur[p] + nc_add : nc_fixed) * nq;
  const int b0 = dboff[p], b1 = dboff[p + 1];
  for (int idx = threadIdx.x; idx < nout; idx += BT) {
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += partial[(int64_t)b * pstride + idx];
    out[(int64_t)p * ostride + idx] = s;
  }
}

void launch_dots_b(const BatchDev& B, int nc_add, int nc_fixed, bool use_k, const double* Au, const double* Al,
                   int nq, const double* Xu, const double* Xl, double* out, int ostride, hipStream_t st) {
  const int* kc = use_k ? B.kcur : nullptr;
#define RIGA_DOTSB(NQ)                                                                                        \
  hipLaunchKernelGGL(k_dots_b<NQ>, dim3(B.ndb), dim3(BT), 0, st, B.db, kc, nc_add, nc_fixed, B.live, Au, Al, \
                     B.ntot, Xu, Xl, B.ntot, B.partial, B.pstride)
  switch (nq) {
    case 1: RIGA_DOTSB(1); break;
    case 2: RIGA_DOTSB(2); break;
    case 3: RIGA_DOTSB(3); break;
    default: RIGA_DOTSB(4); break;
  }
#undef RIGA_DOTSB
  hipLaunchKernelGGL(k_dots_final_b, dim3(B.n), dim3(BT), 0, st, B.dboff, kc, nc_add, nc_fixed, B.live, nq,
                     B.partial, B.pstride, out, ostride);
}

// Z[:, q] -= sum_{c < kcur + nc_add} A[:, c] h_p[c * NQ + q] for up to three pairs.
template <int NQ>
__global__ __launch_bounds__(BT) void k_cgs_update_b(const int4* __restrict__ rb, const int* __restrict__ kcur,
                                                     int nc_add, const unsigned char* __restrict__ live,
                                                     const double* __restrict__ h, int hstride,
                                                     const double* __restrict__ A0, double* __restrict__ Z0,
                                                     const double* __restrict__ A1, double* __restrict__ Z1,
                                                     const double* __restrict__ A2, double* __restrict__ Z2,
                                                     int64_t ld) {
  extern __shared__ double hs[];
  const int4 b = rb[blockIdx.x];
  if (live && !live[b.x]) return;
  const int nc = kcur[b.x] + nc_add;
  const double* hp = h + (int64_t)b.x * hstride;
  for (int k = threadIdx.x; k < nc * NQ; k += BT) hs[k] = hp[k];
  __syncthreads();
  const int64_t i = b.y + threadIdx.x;
  if (i >= b.z) return;
  double z0[NQ], z1[NQ], z2[NQ];
  cgs_update_row<NQ>(i, nc, hs, A0, Z0, A1, Z1, A2, Z2, ld, ld, z0, z1, z2);
}

void launch_cgs_update_b(const BatchDev& B, int nc_add, int nq, const double* h, int hstride, const double* A0,
                         double* Z0, const double* A1, double* Z1, const double* A2, double* Z2, int max_nc,
                         hipStream_t st) {
  const size_t shm = (size_t)max_nc * nq * sizeof(double);
#define RIGA_UPDB(NQ)                                                                                          \
  hipLaunchKernelGGL(k_cgs_update_b<NQ>, dim3(B.nrb), dim3(BT), shm, st, B.rb, B.kcur, nc_add, B.live, h, hstride, \
                     A0, Z0, A1, Z1, A2, Z2, B.ntot)
  switch (nq) {
    case 1: RIGA_UPDB(1); break;
    case 2: RIGA_UPDB(2); break;
    case 3: RIGA_UPDB(3); break;
    default: RIGA_UPDB(4); break;
  }
#undef RIGA_UPDB
}

// Tile passes (bodies in krylov_dev.hpp) per dot block: the block's rows are
// taken in 64-row tiles with nc = kcur + nc_add columns;
// partial[blk * pstride + c * NQ + q] receives the block's products for
// k_dots_final_b.  Products alone: blockIdx.y picks the group of
// CGS_DOT_W * CPW columns.
template <int NQ, int CPW>
__global__ __launch_bounds__(CGS_DOT_W * 64) void k_cgs_dots_b(const int4* __restrict__ db,
                                                               const int* __restrict__ kcur, int nc_add,
                                                               const unsigned char* __restrict__ live,
                                                               const double* __restrict__ Vu,
                                                               const double* __restrict__ Wl,
                                                               const double* __restrict__ Xu,
                                                               const double* __restrict__ Xl, int64_t ld,
                                                               double* __restrict__ partial, int pstride) {
  const int4 b = db[blockIdx.x];
  if (live && !live[b.x]) return;
  const int nc = kcur[b.x] + nc_add;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = ((int)blockIdx.y * CGS_DOT_W + wave) * CPW;
  if (c0 >= nc) return;
  double acc[CPW][NQ];
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] = 0.0;
  for (int64_t r0 = b.y; r0 < b.z; r0 += 64)
    cgs_tile_dots<NQ, CPW>(r0, min((int64_t)b.z, r0 + 64), nc, c0, Vu, Wl, ld, Xu, Xl, ld, lane, acc);
  double* out = partial + (int64_t)blockIdx.x * pstride;
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double v = wave_sum(acc[j][q]);
      if (lane == 0 && c0 + j < nc) out[(c0 + j) * NQ + q] = v;
    }
}

// Update fused with the products: NW waves own NW * CPW columns.
template <int NQ, int NW, int CPW>
__global__ __launch_bounds__(NW * 64) void k_cgs_upd_dots_b(const int4* __restrict__ db,
                                                            const int* __restrict__ kcur, int nc_add,
                                                            const unsigned char* __restrict__ live,
                                                            const double* __restrict__ h, int hstride,
                                                            const double* __restrict__ Vu,
                                                            const double* __restrict__ Vl,
                                                            const double* __restrict__ Wl, double* __restrict__ Zu,
                                                            double* __restrict__ Zl, double* __restrict__ Zw,
                                                            int64_t ld, double* __restrict__ partial, int pstride) {
  __shared__ double hs[NW * CPW * NQ];
  __shared__ double red[NW * 3 * NQ * 64];
  __shared__ double fin[3 * NQ * 64];
  const int4 b = db[blockIdx.x];
  if (live && !live[b.x]) return;   // the whole workgroup leaves together
  const int nc = kcur[b.x] + nc_add;
  const double* hp = h + (int64_t)b.x * hstride;
  for (int k = threadIdx.x; k < NW * CPW * NQ; k += NW * 64) hs[k] = k < nc * NQ ? hp[k] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[CPW][NQ];
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[j][q] = 0.0;
  for (int64_t r0 = b.y; r0 < b.z; r0 += 64)
    cgs_tile_update<NQ, NW, CPW>(r0, min((int64_t)b.z, r0 + 64), nc, hs, Vu, Vl, Wl, ld, Zu, Zl, Zw, ld, red, fin,
                                 lane, wave, acc);
  double* out = partial + (int64_t)blockIdx.x * pstride;
  const int c0 = wave * CPW;
#pragma unroll
  for (int j = 0; j < CPW; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double v = wave_sum(acc[j][q]);
      if (lane == 0 && c0 + j < nc) out[(c0 + j) * NQ + q] = v;
    }
}

template <int NQ>
void launch_cgs_dots_b(const BatchDev& B, bool narrow, int gy, int nc_add, const double* Vu, const double* Wl,
                       const double* Xu, const double* Xl, hipStream_t st) {
  if (narrow)
    hipLaunchKernelGGL((k_cgs_dots_b<NQ, CGS_NARROW_C>), dim3(B.ndb, gy), dim3(CGS_DOT_W * 64), 0, st, B.db, B.kcur,
                       nc_add, B.live, Vu, Wl, Xu, Xl, B.ntot, B.partial, B.pstride);
  else
    hipLaunchKernelGGL((k_cgs_dots_b<NQ, CGS_WIDE_C>), dim3(B.ndb, gy), dim3(CGS_DOT_W * 64), 0, st, B.db, B.kcur,
                       nc_add, B.live, Vu, Wl, Xu, Xl, B.ntot, B.partial, B.pstride);
}

bool launch_cgs_dots_tile_b(const BatchDev& B, int nc_add, int nq, int max_nc, const double* Vu, const double* Wl,
                            const double* Xu, const double* Xl, double* out, int ostride, hipStream_t st) {
  if (!cgs_tile_fits(max_nc, nq)) return false;
  const bool narrow = max_nc <= CGS_NARROW_W * CGS_NARROW_C;
  const int cpw = narrow ? CGS_NARROW_C : CGS_WIDE_C;
  const int gy = (max_nc + CGS_DOT_W * cpw - 1) / (CGS_DOT_W * cpw);
  switch (nq) {
    case 1: launch_cgs_dots_b<1>(B, narrow, gy, nc_add, Vu, Wl, Xu, Xl, st); break;
    case 2: launch_cgs_dots_b<2>(B, narrow, gy, nc_add, Vu, Wl, Xu, Xl, st); break;
    case 3: launch_cgs_dots_b<3>(B, narrow, gy, nc_add, Vu, Wl, Xu, Xl, st); break;
    default: launch_cgs_dots_b<4>(B, narrow, gy, nc_add, Vu, Wl, Xu, Xl, st); break;
  }
  hipLaunchKernelGGL(k_dots_final_b, dim3(B.n), dim3(BT), 0, st, B.dboff, B.kcur, nc_add, 0, B.live, nq, B.partial,
                     B.pstride, out, ostride);
  return true;
}

// The wide shape only for up to two block columns (register budget).
template <int NQ>
void launch_cgs_upd_dots_b(const BatchDev& B, bool narrow, int nc_add, const double* h, int hstride,
                           const double* Vu, const double* Vl, const double* Wl, double* Zu, double* Zl, double* Zw,
                           hipStream_t st) {
  if constexpr (NQ <= 2) {
    if (!narrow) {
      hipLaunchKernelGGL((k_cgs_upd_dots_b<NQ, CGS_WIDE_W, CGS_WIDE_C>), dim3(B.ndb), dim3(CGS_WIDE_W * 64), 0, st,
                         B.db, B.kcur, nc_add, B.live, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, B.ntot, B.partial,
                         B.pstride);
      return;
    }
  }
  hipLaunchKernelGGL((k_cgs_upd_dots_b<NQ, CGS_NARROW_W, CGS_NARROW_C>), dim3(B.ndb), dim3(CGS_NARROW_W * 64), 0,
                     st, B.db, B.kcur, nc_add, B.live, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, B.ntot, B.partial,
                     B.pstride);
}

bool launch_cgs_update_dots_b(const BatchDev& B, int nc_add, int nq, int max_nc, const double* h, int hstride,
                              const double* Vu, const double* Vl, const double* Wl, double* Zu, double* Zl,
                              double* Zw, double* out, int ostride, hipStream_t st) {
  if (!cgs_tile_fits(max_nc, nq)) return false;
  const bool narrow = max_nc <= CGS_NARROW_W * CGS_NARROW_C;
  switch (nq) {
    case 1: launch_cgs_upd_dots_b<1>(B, narrow, nc_add, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, st); break;
    case 2: launch_cgs_upd_dots_b<2>(B, narrow, nc_add, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, st); break;
    case 3: launch_cgs_upd_dots_b<3>(B, narrow, nc_add, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, st); break;
    default: launch_cgs_upd_dots_b<4>(B, narrow, nc_add, h, hstride, Vu, Vl, Wl, Zu, Zl, Zw, st); break;
  }
  hipLaunchKernelGGL(k_dots_final_b, dim3(B.n), dim3(BT), 0, st, B.dboff, B.kcur, nc_add, 0, B.live, nq, B.partial,
                     B.pstride, out, ostride);
  return true;
}

// One workgroup per problem: block_normalize_body with the problem's arrays;
// nc = kcur + nc_add and H column kcur (use_k), or nc = 0 and no H (start block).
__global__ __launch_bounds__(BT) void k_block_normalize_b(const int* __restrict__ kcur, int nc_add,
                                                          const unsigned char* __restrict__ live, int nq,
                                                          const double* h1, const double* h2, int hstride,
                                                          const double* G, double* H, int ldh,
                                                          double* Rinv, int* flag) {
  __shared__ double hn[4];
  const int p = blockIdx.x;
  if (live && !live[p]) return;
  const int nc = kcur ? kcur[p] + nc_add : 0;
  const int k = kcur ? kcur[p] : 0;
  block_normalize_body(nc, nq, nc > 0 ? h1 + (int64_t)p * hstride : nullptr,
                       nc > 0 ? h2 + (int64_t)p * hstride : nullptr, G + (int64_t)p * nq * nq,
                       H ? H + (int64_t)p * ldh * ldh : nullptr, ldh, k, Rinv + (int64_t)p * nq * nq, flag + p, hn);
}

void launch_block_normalize_b(const BatchDev& B, bool use_k, int nc_add, int nq, const double* h1,
                              const double* h2, int hstride, const double* G, double* H, int ldh, double* Rinv,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_block_normalize_b, dim3(B.n), dim3(BT), 0, st, use_k ? B.kcur : nullptr, nc_add, B.live, nq,
                     h1, h2, hstride, G, H, ldh, Rinv, B.flag);
}

// Out_m[:, col + c] = sum_a In_m[:, a] Rinv_p[a][c], col = kcur + col_add (or col_add).
template <int NQ>
__global__ __launch_bounds__(BT) void k_gemm3_b(const int4* __restrict__ rb, const int* __restrict__ kcur,
                                                int col_add, const unsigned char* __restrict__ live,
                                                const double* __restrict__ Rinv, const double* __restrict__ I0,
                                                double* __restrict__ O0, const double* __restrict__ I1,
                                                double* __restrict__ O1, const double* __restrict__ I2,
                                                double* __restrict__ O2, int64_t ld) {
  const int4 b = rb[blockIdx.x];
  if (live && !live[b.x]) return;
  const int64_t i = b.y + threadIdx.x;
  if (i >= b.z) return;
  const int64_t col = (kcur ? kcur[b.x] : 0) + col_add;
  const double* Q = Rinv + (int64_t)b.x * NQ * NQ;
  double q[NQ][NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a)
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[a][c] = Q[a + c * NQ];
  const double* Is[3] = {I0, I1, I2};
  double* Os[3] = {O0, O1, O2};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double x[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a) x[a] = Is[m][i + a * ld];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < NQ; ++a) acc += x[a] * q[a][c];
      Os[m][i + (col + c) * ld] = acc;
    }
  }
}

void launch_gemm3_b(const BatchDev& B, bool use_k, int col_add, int nq, const double* Rinv, const double* I0,
                    double* O0, const double* I1, double* O1, const double* I2, double* O2, hipStream_t st) {
  const int* kc = use_k ? B.kcur : nullptr;
#define RIGA_G3B(NQ)                                                                                            \
  hipLaunchKernelGGL(k_gemm3_b<NQ>, dim3(B.nrb), dim3(BT), 0, st, B.rb, kc, col_add, B.live, Rinv, I0, O0, I1, O1, \
                     I2, O2, B.ntot)
  switch (nq) {
    case 1: RIGA_G3B(1); break;
    case 2: RIGA_G3B(2); break;
    case 3: RIGA_G3B(3); break;
    default: RIGA_G3B(4); break;
  }
#undef RIGA_G3B
}

// End of a block step: live problems move to the next block; a problem stays
// live while another block fits in the subspace of size m.
__global__ void k_advance_b(int n, int b, int m, int* __restrict__ kcur, unsigned char* __restrict__ live) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    if (!live[p]) continue;
    const int k = kcur[p] + b;
    kcur[p] = k;
    live[p] = (k + b <= m) ? 1 : 0;
  }
}

void launch_advance_b(const BatchDev& B, int b, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_b, dim3((B.n + 255) / 256), dim3(256), 0, st, B.n, b, m, B.kcur, B.live);
}

// Out[:, 0:kout_p] = In[:, 0:kin_p] Q_p per problem (Q_p at Q + qoff[p], kin_p x
// kout_p column-major); problems with kout_p = 0 are skipped.  A row block of up
// to 256 rows is done as 64-row tiles.
// Outputs of at most 32 columns from at most 128 inputs in every problem (the
// usual short bases of the batched form) take the LDS tile, otherwise the
// matrix cores; separate kernels, so each keeps its own register budget.
constexpr int GEMM_NARROW_OUT = 32, GEMM_NARROW_IN = 128;

__global__ __launch_bounds__(256) void k_gemm_tall_b_tile(const int4* __restrict__ rb,
                                                          const int* __restrict__ kin,
                                                          const int* __restrict__ kout,
                                                          const int64_t* __restrict__ qoff,
                                                          const double* __restrict__ Q,
                                                          const double* __restrict__ In, double* __restrict__ Out,
                                                          int64_t ld) {
  extern __shared__ double qs[];
  const int4 b = rb[blockIdx.x];
  const int ko = kout[b.x];
  if (ko <= 0) return;
  for (int r0 = b.y; r0 < b.z; r0 += 64)
    gemm_tile64(r0, min(64, b.z - r0), In, ld, kin[b.x], Q + qoff[b.x], ko, Out, ld, qs);
}

__global__ __launch_bounds__(256) void k_gemm_tall_b(const int4* __restrict__ rb,
                                                     const int* __restrict__ kin,
                                                     const int* __restrict__ kout,
                                                     const int64_t* __restrict__ qoff,
                                                     const double* __restrict__ Q,
                                                     const double* __restrict__ In, double* __restrict__ Out,
                                                     int64_t ld) {
  extern __shared__ double qs[];
  const int4 b = rb[blockIdx.x];
  const int ko = kout[b.x];
  if (ko <= 0) return;
  // a row block holds at most 256 rows: four 16-row slabs for each of 4 waves
  gemm_rows_mfma<4, 4>(b.y, b.z, In, ld, kin[b.x], Q + qoff[b.x], ko, Out, ld, qs);
}

void launch_gemm_tall_b(const BatchDev& B, const int* kin, const int* kout, const int64_t* qoff, const double* Q,
                        int max_kin, int max_kout, const double* In, double* Out, hipStream_t st) {
  if (max_kout <= GEMM_NARROW_OUT && max_kin <= GEMM_NARROW_IN) {
    const size_t shm = (size_t)max_kin * 80 * sizeof(double);
    hipLaunchKernelGGL(k_gemm_tall_b_tile, dim3(B.nrb), dim3(256), shm, st, B.rb, kin, kout, qoff, Q, In, Out,
                       B.ntot);
  } else {
    const size_t shm = (size_t)gemm_lds_doubles(max_kin) * sizeof(double);
    hipLaunchKernelGGL(k_gemm_tall_b, dim3(B.nrb), dim3(256), shm, st, B.rb, kin, kout, qoff, Q, In, Out, B.ntot);
  }
}

}  // namespace riga
