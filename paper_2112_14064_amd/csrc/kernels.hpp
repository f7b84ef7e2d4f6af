// Launchers of the gfx950 kernels (host side).  Every pointer is device memory
// unless stated otherwise; every launch is asynchronous on `st`.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>
#include <cstdint>

namespace riga {

// Device copy of the 1-D space and of the nested-dissection plan.
struct DevSpace {
  int p, ne, n;                 // degree, elements, Dirichlet functions per direction
  const int* knots;             // element-boundary indices, length nall + p + 1
  const int* sup0; const int* sup1;
  const int* lo; const int* hi;
  const int* first;             // per element
  const int64_t* rowptr;        // CSR row pointers (ndof + 1)
  // explicit CSR column indices (vector spaces), or null: the scalar space's
  // columns are implicit in lo / hi (tensor pattern)
  const int* col;
};

struct DevTree {
  const int* nf; const int* no; const int* nb;
  const int64_t* loff; const int64_t* uoff;
  const int* foff; const int* fdofs; const int* fkey; const int* fpos;
  const int* coff; const int* clist; const int* moff; const int* maps;
  const int* voff;              // per node: offset of its solve update vector (nb entries)
  // Forward-sweep gather lists: front position foff[v] + p receives the update
  // rows gidx[gptr[foff[v] + p] .. gptr[foff[v] + p + 1]) (rows of the update
  // array, children in clist order), so a front is assembled without a pass
  // per child.
  const int* gptr; const int* gidx;
  // per front position foff[v] + p: {its dof for p < no, else -1; number of
  // update rows; the first of them; the second of them when there are two,
  // else the list's index in gidx}
  const int4* gsrc;
  const int64_t* doff;          // per node: first 64x64 block of its diagonal inverses
  const unsigned char* prec;    // per node: 1 = FP32 front (mixed factor), or null (all FP64)
  const int64_t* lpoff;         // per node: sweep layouts of F (see lp_group / tp_group;
  const int64_t* tpoff;         //   room for groups of 2 and of 4 elements)
  double* sgn;                  // per dof: sign of its pivot in the signed factorization
                                //   K - s M = L S L^T (null: Cholesky, every sign +1)
  const unsigned char* ttri;    // per node: 1 = Tp without the zero triangle, 0 = full
                                //   rectangle (F[gK + s][a] at ((g no + a) K + s))
  // Forest of independent problems (batched form), all null for one problem:
  const int* inst;              // per node: its problem
  const DevSpace* spaces;       // per problem: 1-D space, rowptr into the forest CSR rows
  const int64_t* dofbase;       // per problem: first dof in the forest numbering
  const double* isig;           // per problem: shift sigma
  const unsigned char* ilive;   // per problem: 0 = skip its nodes in the sweeps (may be null)
};

// --- assembly ---------------------------------------------------------------
// 1-D element mass / stiffness blocks tabM/tabK[e][a][b], a,b in 0..p, from
// the Cox--de Boor values at the (p+1)-point Gauss rule (gx, gw on [-1, 1]);
// tabS (may be null) the blocks of int B_a dB_b/dx.
void launch_bspline_tables(const DevSpace& s, const double* gx, const double* gw,
                           double* tabM, double* tabK, double* tabS, hipStream_t st);
// Band of the 1-D skew matrix s_ij = int B_i B_j' from tabS (layout of M1).
void launch_band_skew(const DevSpace& s, const double* tabS, double* S1, hipStream_t st);
// Banded 1-D factors of M and K of a space (see k_assemble.hip): M1, K1 hold
// n (2p + 1) doubles, entry (i, ii) at i (2p + 1) + ii - i + p.
void launch_band_1d(const DevSpace& s, const double* tabM, const double* tabK, double* M1, double* K1,
                    hipStream_t st);
// CSR values of K, M and C = alpha M + beta K + sum_e c_e M_e from the bands
// (launch_band_1d first) and, for c_elem, the element tables: one wave per row.
// With S1 (launch_band_skew) C also gets the gyroscopic part
// gx M1 (x) S1 + gy S1 (x) M1 (x fastest) and Ct the values of C^T.
void launch_assemble(const DevSpace& s, const double* tabM, const double* M1, const double* K1,
                     double alpha, double beta, const double* c_elem,
                     double* K, double* M, double* C, int64_t ndof, hipStream_t st,
                     const double* S1 = nullptr, double gx = 0.0, double gy = 0.0, double* Ct = nullptr);
// K, M, C = alpha M + beta K of the H(curl) space (see k_assemble.hip) from
// the dense 1-D matrices MA (na x na), MB, KB (nb x nb), D (na x nb); rows
// from base1 on are component 1.
void launch_assemble_hcurl(int na, int nb, int64_t base1, int64_t ndof, const int64_t* rowptr, const int* col,
                           const double* MA, const double* MB, const double* KB, const double* D, double alpha,
                           double beta, double* K, double* M, double* C, hipStream_t st);
// Divergence-conforming space (see k_assemble.hip): K = div-div + alpha G,
// M, C = beta G with G the absorbing walls' normal-component integral (walls:
// bits left, right, bottom, top); 1-D matrices of A (na) and of the x / y
// degree-p spaces (nbx, nby kept functions).
void launch_assemble_hdiv(int na, int nbx, int nby, int64_t base1, int64_t ndof, const int64_t* rowptr,
                          const int* col, const double* MA, const double* MBx, const double* KBx, const double* Dx,
                          const double* MBy, const double* KBy, const double* Dy, int walls, double alpha,
                          double beta, double* K, double* M, double* C, hipStream_t st);
// Bands of every problem of a forest: problem q's tables at taboff[q], its
// bands at bandoff[q] (max_w: the largest n (2p + 1)).
void launch_band_1d_b(const DevSpace* spaces, int n, int max_w, const int64_t* taboff, const double* tabM,
                      const double* tabK, const int64_t* bandoff, double* M1, double* K1, hipStream_t st);
// Tables, bands and entries for every problem of a forest in three launches:
// per problem q its space spaces[q], first row dofbase[q], tables at tabM/tabK
// + taboff[q], bands at M1/K1 + bandoff[q], Gauss rule gx[q]/gw[q] (device
// pointer arrays), damping alpha[q], beta[q], c_elem[q] (may be null); rb: row
// blocks of at most 256 rows of one problem.
void launch_assemble_b(const int4* rb, int nrb, const DevSpace* spaces, const int64_t* dofbase,
                       const int64_t* taboff, const double* const* gx, const double* const* gw, int n, int max_ne,
                       double* tabM, double* tabK, int max_w, const int64_t* bandoff, double* M1, double* K1,
                       const double* alpha, const double* beta, const double* const* c_elem, double* K, double* M,
                       double* C, hipStream_t st);

// --- factorization ------------------------------------------------------------
// One tree level: assemble each front (original entries of Q = s2 M + s1 C + K
// plus the children's update blocks), eliminate its own dofs by a 64-wide
// blocked right-looking Cholesky with MFMA panel and trailing updates, and
// leave F = [L_oo^{-1}; L_bo L_oo^{-1}] column-major in L (nf x no per node)
// and F in the sweep layouts Lp (lpoff: groups of 16 bytes of columns) and
// Tp (tpoff: groups of rows); L, U, T are working storage of the
// factorization.  D holds the 64x64 inverses of the diagonal blocks (doff);
// max_no / max_nf bound the level, max_child_nb / max_kids its children.
// FP64 level: children flagged in t.prec keep their update blocks in U32.
// One tree level of the LU factorisation of a nonsymmetric Q = s2 M + s1 C + K
// (C with a skew part; Ct: the values of C^T on the same pattern) without
// pivoting (see k_factor.hip): the front of A in L / U with the factor L in Lx
// and its diagonal-block inverses in D, the front of A^T in R / UR with the
// transposed upper factor in Rx and inverses in DR; the forward sweep layout
// Lp from L's F and the backward layout Tp from Ut's F.  FP64 only.
void launch_front_factor_lu(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                            int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K,
                            const double* M, const double* C, const double* Ct, double* L, double* U, double* Lx,
                            double* D, double* R, double* UR, double* Rx, double* DR, double* Lp, double* Tp,
                            int64_t* status, hipStream_t st);
void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                         int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                         const double* C, double* L, double* U, double* T, double* D, double* Lp, double* Tp,
                         const float* U32, int64_t* status, hipStream_t st);
// FP32 level (FP32 products and accumulation); all children are FP32.
void launch_front_factor(const DevSpace& s, const DevTree& t, const int* level_nodes, int count, int max_no,
                         int max_nf, int max_child_nb, int max_kids, double s2, double s1, const double* K, const double* M,
                         const double* C, float* L, float* U, float* T, float* D, float* Lp, float* Tp,
                         int64_t* status, hipStream_t st);
// Out = am M + ac C + ak K on the shared CSR pattern (nnz values).
void launch_combine3(int64_t nnz, double am, const double* M, double ac, const double* C, double ak,
                     const double* K, double* Out, hipStream_t st);

// --- forward / backward solves ------------------------------------------------
// One launch per tree level; tasks[k] = {node, first row, end row, 0}.  The
// level's factor is read in its sweep layouts, FP64 (Lp64/Tp64) or FP32
// (Lp32/Tp32 non-null).
// Sweep layouts of F = [L_oo^{-1}; L_bo L_oo^{-1}] (nf x no) without the zero
// triangle of L_oo^{-1}, in groups of K side-by-side entries (one 16-byte load):
//   forward (Lp): group g of columns gK .. gK+K-1 holds rows gK .. nf-1 (the
//     rows above are zeros), row r at lp_group(g) + r - gK (in groups);
//   backward (Tp): group g of rows gK .. gK+K-1 holds columns
//     0 .. tp_width(g)-1 (the columns right of the diagonal block are zeros),
//     column a at tp_group(g) + a.  Only nodes of levels with many backward
//     tasks use it (the leaves, where the triangle is a large share of F and
//     the sweep is bandwidth-bound); the others keep the full rectangle.
__host__ __device__ inline int64_t lp_group(int g, int nf, int K) {
  return (int64_t)g * nf - (int64_t)K * g * (g - 1) / 2;
}
__host__ __device__ inline int tp_width(int g, int no, int K) { return (g + 1) * K < no ? (g + 1) * K : no; }
__host__ __device__ inline int64_t tp_group(int g, int no, int K) {
  const int g1 = (no + K - 1) / K;   // groups below g1 - 1 are (g + 1) K wide, later ones no
  if (g < g1) return (int64_t)K * g * (g + 1) / 2;
  return (int64_t)K * (g1 - 1) * g1 / 2 + (int64_t)(g - g1 + 1) * no;
}
// Entries of a node's layouts for groups of K.
__host__ __device__ inline int64_t lp_size(int nf, int no, int K) { return K * lp_group((no + K - 1) / K, nf, K); }
__host__ __device__ inline int64_t tp_size(int nf, int no, int K) { return K * tp_group((nf + K - 1) / K, no, K); }

// One task of a sweep level: rows [r0, r1) of F of node v (forward) or own
// columns [r0, r1) (backward), with the node fields the workgroup needs, so
// that it starts from a single load.  poff: the node's lpoff (forward) or
// tpoff (backward); inst: the node's problem in a forest, else 0.
struct alignas(16) SweepTask {
  int v, r0, r1, nf;
  int no, foff, voff, inst;
  int64_t poff, unused;
};
// `variant` selects the task tile shape (0 .. sweep_variants()-1, see sweep_variant);
// max_front bounds the fronts of the given tasks (it sizes the shared memory of
// a workgroup, so the level's own largest front keeps occupancy up).
void launch_fwd_level(const DevTree& t, const SweepTask* tasks, int count, int nrhs, const double* Lp64,
                      const float* Lp32, const double* b, int64_t ldb, double* y, int64_t ldy, double* upd,
                      int max_front, int variant, hipStream_t st);
int sweep_variants();
// Variant a level starts from before any autotuning, by its task count:
// levels with many tasks (bandwidth-bound) take 4-wave tasks, middle levels 8
// waves with short rounds, and the few-task levels near the root (a task's
// rows stream from one compute unit) 16 waves, so more loads are in flight
// per task.
int sweep_default_variant(int tasks, bool forward);
// Levels with at least this many backward tasks keep the backward layout
// without the zero triangle (build_sweep_plan packs them so, launch_bwd_level
// reads them so).
constexpr int SWEEP_TRI_TASKS = 1024;
// Waves per task and column groups per wave and round of a sweep variant.
void sweep_variant(int v, int* waves, int* groups);
// Outputs of the backward sweep (see k_bwd): xs holds the sweep's solution
// (negated if neg), optionally ru = scale (x + base) and rl = sig val + v_u.
struct BwdOut {
  double* xs = nullptr; int64_t ldxs = 0; int neg = 0;
  const double* base = nullptr; int64_t ldbase = 0;
  double* ru = nullptr; int64_t ldr = 0; double scale = 1.0;
  double* rl = nullptr; const double* v_u = nullptr; int64_t ldv = 0; double sig = 0.0;
};
void launch_bwd_level(const DevTree& t, const SweepTask* tasks, int count, int nrhs, const double* Tp64,
                      const float* Tp32, const double* y, int64_t ldy, const BwdOut& o, int max_front, int variant,
                      hipStream_t st);

// --- Krylov building blocks -----------------------------------------------------
// Sliced-ELL copy of a CSR value array for the Krylov products: slabs of 64
// consecutive rows of one problem; entry o of the slab's row r0 + l at
// E[off + 64 o + l] for o < width (the slab's longest row; shorter rows padded
// with zeros).  Columns stay implicit in the tensor structure.
struct alignas(16) EllSlab {
  int inst, r0, nrows, width;   // problem (0 for one problem), first row (global), rows, entries per row
  int64_t off;
};
// Slabs of the rows [r0, r1) of problem inst for every range; returns the
// entries of the layout.
int64_t build_ell_slabs(const std::vector<int64_t>& rowptr, const std::vector<int4>& ranges,
                        std::vector<EllSlab>& slabs);
void launch_csr_to_ell(const EllSlab* slabs, int nslab, const int64_t* rowptr, const double* V, double* E,
                       hipStream_t st);
// Y = E X + bz Z (Z may be null) on the slabs' rows (of live problems when
// live is not null): spaces[inst] and dofbase[inst] (null: 0) locate a slab's
// problem.  ncols <= 4; a workgroup per slab, lane = row, its 4 waves taking
// interleaved rounds of 7 entries whose loads are in flight together.
void launch_spmv_ell(const EllSlab* slabs, int nslab, const DevSpace* spaces, const int64_t* dofbase,
                     const unsigned char* live, int ncols, const double* E, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, const double* Z, int64_t ldz, double bz, hipStream_t st);
// Y = a A X + bz Z (Z may be null) and optionally Y2 = A X.  X, Y, Z, Y2:
// ndof x ncols (ld given), ncols <= 8.
void launch_spmv(const DevSpace& s, int64_t ndof, int ncols, const double* A, double a, const double* X,
                 int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz, double bz, double* Y2,
                 int64_t ldy2, hipStream_t st);
// Y0 = A0 X, Y1 = A1 X, Y2 = A2 X in one pass over X (ncols <= 8, common ld of the Y);
// explicit columns when s.col is set (vector spaces), else the tensor pattern.
void launch_spmv3(const DevSpace& s, int64_t ndof, int ncols, const double* A0, const double* A1, const double* A2,
                  const double* X, int64_t ldx, double* Y0, double* Y1, double* Y2, int64_t ldy, hipStream_t st);
// out[c*nq + q] = sum_i Au[i,c] Xu[i,q] + Al[i,c] Xl[i,q]  (Al/Xl may be null),
// c < nc, q < nq <= 4; deterministic two-stage reduction.  partial: >= nblk*nc*nq
// doubles of scratch.
void launch_dots(int64_t n, int nc, const double* Au, const double* Al, int64_t lda,
                 int nq, const double* Xu, const double* Xl, int64_t ldx,
                 double* partial, double* out, hipStream_t st);
int dots_blocks(int64_t n);
// out[o] = sum over the nblk partial sums partial[o nblk + b] (second stage of
// the products above, one wave per output, fixed order).
void launch_dots_final(int nout, int nblk, const double* partial, double* out, hipStream_t st);
// Z[:, q] -= sum_c A[:, c] h[c*nq+q] for up to three (A, Z) pairs sharing h.
// With gpart (nq <= 4), every block also writes the sum over its rows of the
// updated Z0^T Z0 + Z2^T Z1 (nq x nq) to gpart[block * nq * nq ...]; returns
// the number of blocks.
int launch_cgs_update(int64_t n, int nc, int nq, const double* h,
                      const double* A0, double* Z0, const double* A1, double* Z1,
                      const double* A2, double* Z2, int64_t lda, int64_t ldz, double* gpart, hipStream_t st);
// Pass 1 update of classical Gram--Schmidt fused with the pass 2 products
// (tile kernel, one read of the basis): for the basis (Vu, Vl, Wl; nc columns,
// ld lda) and the block (Zu, Zl, Zw = M Zl; nq columns, ld ldz),
//   Z -= V h for (Vu, Zu), (Vl, Zl), (Wl, Zw), h[c nq + q] on the device, then
//   out[c nq + q] = Vu[:, c]^T Zu[:, q] + Wl[:, c]^T Zl[:, q] of the updated block.
// Returns the number of workgroups, or -1 (nothing launched) when
// cgs_tile_fits(nc, nq) is false.  partial: >= blocks * nc * nq doubles of scratch.
constexpr int CGS_NARROW_W = 4, CGS_NARROW_C = 8;   // waves, columns per wave: nc <= 32
constexpr int CGS_WIDE_W = 8, CGS_WIDE_C = 12;      // nc <= 96 (nq <= 2)
constexpr int CGS_MAX_BLOCKS = 256;   // one workgroup per compute unit, all resident
constexpr int CGS_DOT_W = 4;          // batched products alone: waves per workgroup
// nc <= 96 with nq <= 2, or nc <= 32 with nq <= 4 (the register budget)
bool cgs_tile_fits(int nc, int nq);
int launch_cgs_update_dots(int64_t n, int nc, int nq, const double* h, const double* Vu, const double* Vl,
                           const double* Wl, int64_t lda, double* Zu, double* Zl, double* Zw, int64_t ldz,
                           double* partial, double* out, hipStream_t st);
// Block Gram--Schmidt with the second pass delayed by one step (block nb <= 2;
// the basis Vu, Vl, Wl = M Vl holds the finished columns 0..k and the pending
// block Y at k..k+nb, projected once and not normalised; W = (Ru, Rl, MRl) the
// operator applied to Y):
//   launch_dcgs_dots    out = [V Y]^T_B [Y W] ((k+nb) x 2nb output-major; only
//                       [V Y]^T_B Y without W) and, with s, MRl = M Rl on the
//                       tensor grid in the same launch;
//   launch_dcgs_coef    one workgroup: the coefficients hc ((k+nb) x 2nb, or
//                       x nb), Xm = T^{-1} (nb x nb), H's new column block
//                       (rows 0..k+2nb of columns k..k+nb) and its columns 0..k
//                       rewritten for the finished block; a block in the span
//                       of V sets *flag;
//   launch_dcgs_update  Y finished in place and, with W, the projected image
//                       W Xm - [V Y] hc written to V[:, k+nb:k+2nb] as the next
//                       pending block.
void launch_dcgs_dots(int64_t n, int k, int nb, bool hasw, const double* Vu, const double* Vl, const double* Wl,
                      int64_t lda, const double* Ru, const double* Rl, double* partial, double* out,
                      const DevSpace* s, const double* M1, double* MRl, hipStream_t st);
void launch_dcgs_coef(int k, int nb, bool hasw, const double* P, double* H, int ldh, double* hc, double* Xm,
                      int* flag, hipStream_t st);
void launch_dcgs_update(int64_t n, int k, int nb, bool hasw, const double* hc, const double* Xm, double* Vu,
                        double* Vl, double* Wl, int64_t lda, const double* Zu, const double* Zl, const double* Zw,
                        int64_t ldz, hipStream_t st);
// Y = a M X + b K X + c Z on the tensor grid of a space (X[j n + i], nq <= 4
// columns; Z may be null) by sum factorisation with the banded 1-D factors:
// per 64 x 8 tile of the grid, T = X M1^T and X K1^T along i, then
// Y = M1 (a T_M + b T_K) + b K1 T_M along j, all in shared memory.  Reads X
// with a halo of p rows and columns instead of the stored entries of the
// 2-D matrices.
void launch_tensor_mk(const DevSpace& s, const double* M1, const double* K1, int nq, double a, double b,
                      const double* X, int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz, double c,
                      hipStream_t st);
// Grid tiles of the sum-factorised product (64 along i, 8 along j).
constexpr int TENSOR_TILE_I = 64, TENSOR_TILE_J = 8;
// Forest form of launch_tensor_mk: tiles[t] = {problem, i0, j0, 0} over the
// grids of every problem (problem q's rows start at dofbase[q], its bands at
// M1 / K1 + bandoff[q]); Y = (sig + alpha) M X + beta K X + c Z per problem, or
// with sig null Y = M X + c Z.  Problems with live[q] == 0 are skipped; max_p
// bounds the degrees (shared memory size).
void launch_tensor_mk_b(const int4* tiles, int ntiles, const DevSpace* spaces, const int64_t* dofbase,
                        const int64_t* bandoff, const double* M1, const double* K1, const unsigned char* live,
                        const double* sig, const double* alpha, const double* beta, int nq, int max_p,
                        const double* X, int64_t ldx, double* Y, int64_t ldy, const double* Z, int64_t ldz,
                        double c, hipStream_t st);
// Out[i + c ldo] = sum_t In[i + t ldi] Q[t, c] (Q device, kin x kout col-major,
// kin <= 254), on the FP64 matrix cores.
void launch_gemm_tall(int64_t n, const double* In, int64_t ldi, int kin, const double* Q, int kout,
                      double* Out, int64_t ldo, hipStream_t st);
// Counter-based uniform(-1, 1) fill of a ndof x ncols block (splitmix64 of seed, index).
void launch_random_fill(double* X, int64_t n, int ncols, int64_t ld, uint64_t seed, hipStream_t st);
// Eigenvector post-processing on planar complex columns P = [a_1..a_nv | b_1..b_nv]
// (ld rows each) with MP = M P, CP = C P, KP = K P; see k_krylov.hip.
void launch_pair_forms(int64_t n, int nv, const double* P, const double* MP, const double* CP,
                       const double* KP, int64_t ld, double* part, int nsplit, hipStream_t st);
// b_k^T (C a_k) of every planar pair (see k_krylov.hip): part[k nsplit + x].
void launch_cross_form(int64_t n, int nv, const double* P, const double* CP, int64_t ld, double* part, int nsplit,
                       hipStream_t st);
void launch_pair_resid(int64_t n, int nv, const double* P, const double* MP, const double* CP,
                       const double* KP, int64_t ld, const double* lam, double* part, int nsplit,
                       hipStream_t st);
void launch_finalize(int64_t n, int nv, int nout, const double* P, int64_t ld, const double* s, double* X,
                     hipStream_t st);
// Largest absolute row sums of A0, A1, A2 (shared rowptr) per block of rows:
// part[3 b + a].  Blocks are rb[b] = {problem, first row, end row, 0} (forest)
// or, with rb null, consecutive runs of rows_per_block rows of ndof.
void launch_rowabs3(const int4* rb, int nblocks, int64_t ndof, int rows_per_block, const int64_t* rowptr,
                    const double* A0, const double* A1, const double* A2, double* part, hipStream_t st);

// launch_dots (nc > 0) together with M1 (x) M1 applied to the nq columns of
// Xl (the space s, ldx) into Y2: one launch for both, then the final sums.
void launch_dots_mr(int64_t n, int nc, const double* Au, const double* Al, int64_t lda, int nq, const double* Xu,
                    const double* Xl, int64_t ldx, double* partial, double* out, const DevSpace& s,
                    const double* M1, double* Y2, int64_t ldy2, hipStream_t st);
// Device-side block normalisation fused with the new basis block (see
// k_krylov.hip): H columns k..k+nq from the projection coefficients h1 + h2 and
// the Cholesky factor R of the Gram matrix G (or, with gpart, of the sum of
// gblk partial Gram matrices); Out_m = In_m R^{-1} (n x nq) for up to three
// pairs sharing ld (I1/O1 and I2/O2 may be null); *flag = 1 when a column was
// lost (breakdown).  rbuf: nq x nq device scratch (used when gblk is large).
void launch_normalize_gemm3(int64_t n, int nc, int nq, const double* h1, const double* h2, const double* G,
                            const double* gpart, int gblk, double* H, int ldh, int k, int* flag, double* rbuf,
                            const double* I0, double* O0, const double* I1, double* O1, const double* I2,
                            double* O2, int64_t ld, hipStream_t st);

// Interleaved complex columns -> planar [Re | Im].
void launch_deinterleave(int64_t n, int nv, const double* X, double* P, hipStream_t st);
// grad[e] = sum_k Re(w_k u_k^T M_e u_k) for every element e (see k_krylov.hip).
void launch_adjoint(const DevSpace& s, const double* tabM, int nv, const double* P, int64_t ndof,
                    const double* w, double* grad, hipStream_t st);

// --- batched form (k_batch.hip) ---------------------------------------------
// Device view of a forest of independent problems run in lockstep.
struct BatchDev {
  int n = 0;                        // problems
  int64_t ntot = 0;                 // forest rows (sum of the problems' dofs)
  const int* rinst = nullptr;       // per row: its problem
  const DevSpace* spaces = nullptr; // per problem
  const int64_t* dofbase = nullptr; // per problem: first row
  const double* sig = nullptr;      // per problem: shift
  unsigned char* live = nullptr;    // per problem: takes part in the current step
  int* kcur = nullptr;              // per problem: first column of the current block
  int* flag = nullptr;              // per problem: breakdown flag of the normalisation
  const int4* rb = nullptr;         // row blocks of <= 256 rows, one problem each
  int nrb = 0;
  const int4* db = nullptr;         // dot blocks (longer row ranges, one problem each)
  int ndb = 0;
  const int* dboff = nullptr;       // per problem: its dot blocks [dboff[p], dboff[p+1])
  double* partial = nullptr;        // dot partial sums, pstride per dot block
  int pstride = 0;
};
// A = sigma_p M + C per problem (nonzeros of problem p in [nzbase[p], nzbase[p+1])).
void launch_combine_b(int n, const int64_t* nzbase, int64_t nnz, const double* sig, const double* M, const double* C,
                      double* A, hipStream_t st);
// Current block of the bases (columns kcur .. kcur + nq) into Xu, Xw.
void launch_gather_b(const BatchDev& B, int nq, const double* Vu, const double* Wl, double* Xu, double* Xw,
                     hipStream_t st);
// out[p * ostride + c * nq + q] = A_p[:, c]^T X_p[:, q] (u and l parts), c < nc with
// nc = kcur + nc_add (use_k) or nc_fixed.
void launch_dots_b(const BatchDev& B, int nc_add, int nc_fixed, bool use_k, const double* Au, const double* Al,
                   int nq, const double* Xu, const double* Xl, double* out, int ostride, hipStream_t st);
// Z[:, q] -= A[:, 0:kcur+nc_add] h_p for up to three pairs (max_nc bounds kcur + nc_add).
void launch_cgs_update_b(const BatchDev& B, int nc_add, int nq, const double* h, int hstride, const double* A0,
                         double* Z0, const double* A1, double* Z1, const double* A2, double* Z2, int max_nc,
                         hipStream_t st);
// Batched tile passes on every live problem's dot blocks with
// nc = kcur + nc_add <= max_nc columns; out[p * ostride + c * nq + q]:
//   launch_cgs_dots_tile_b      Vu[:, c]^T Xu[:, q] + Wl[:, c]^T Xl[:, q];
//   launch_cgs_update_dots_b    the fused update and products of
//                               launch_cgs_update_dots with the problem's h
//                               (h + p * hstride).
// Both return false (nothing launched) when cgs_tile_fits(max_nc, nq) is false.
bool launch_cgs_dots_tile_b(const BatchDev& B, int nc_add, int nq, int max_nc, const double* Vu, const double* Wl,
                            const double* Xu, const double* Xl, double* out, int ostride, hipStream_t st);
bool launch_cgs_update_dots_b(const BatchDev& B, int nc_add, int nq, int max_nc, const double* h, int hstride,
                              const double* Vu, const double* Vl, const double* Wl, double* Zu, double* Zl,
                              double* Zw, double* out, int ostride, hipStream_t st);
void launch_block_normalize_b(const BatchDev& B, bool use_k, int nc_add, int nq, const double* h1,
                              const double* h2, int hstride, const double* G, double* H, int ldh, double* Rinv,
                              hipStream_t st);
void launch_gemm3_b(const BatchDev& B, bool use_k, int col_add, int nq, const double* Rinv, const double* I0,
                    double* O0, const double* I1, double* O1, const double* I2, double* O2, hipStream_t st);
void launch_advance_b(const BatchDev& B, int b, int m, hipStream_t st);
void launch_gemm_tall_b(const BatchDev& B, const int* kin, const int* kout, const int64_t* qoff, const double* Q,
                        int max_kin, int max_kout, const double* In, double* Out, hipStream_t st);

// --- compact (TOAR) basis (k_toar.hip) ----------------------------------------
// Z -= U h (n x nq, h[c nq + q] on the device, c < nc) fused with
// out[c nq + q] = U[:, c]^T Z[:, q] of the updated block: one read of U.
// Returns the number of workgroups, or -1 (nothing launched) when
// toar_tile_fits(nc, nq) is false.  partial: >= blocks nc nq doubles.
bool toar_tile_fits(int nc, int nq);
int launch_toar_update_dots(int64_t n, int nc, int nq, const double* h, const double* U, int64_t ldu, double* Z,
                            int64_t ldz, double* partial, double* out, hipStream_t st);
// The compact step of one block (see k_toar.hip): orthogonalise the
// coordinates of the operator's image against the compact basis (Q1, Q2;
// ldq rows), write H's column block k..k+nq, the new basis columns and their
// packed copy P.  false (nothing launched) when the sizes exceed the kernel's
// shared-memory tables (r + nq <= 264, k + nq <= 260, r + nq <= ldq).
bool launch_toar_compact(int r, int k, int nq, double sig, const double* S, int lds, double* Q1, double* Q2, int ldq,
                         double* H, int ldh, int* flag, double* P, hipStream_t st);

// Complex target shift sigma = a + ib (see k_cshift.hip).  Real form of
// -i Q(sigma) on the doubled pattern of Plan::build_realform from the base
// CSR values (n base rows): Kr = J (x) I, Cr = R (x) E, Ctr = -Cr.
void launch_realform_values(int64_t n, const int64_t* rowptr, const double* K, const double* M, const double* C,
                            double a, double b, double* Kr, double* Cr, double* Ctr, hipStream_t st);
// Real-form right-hand sides (2n x nb, ld ldo) of x = -Q^{-1} t from MX = M v_u
// and CW = C v_u + M v_l (n x nb, ld ld).
void launch_cshift_rhs(int64_t n, int nb, const double* MX, const double* CW, int64_t ld, double a, double b,
                       double* out, int64_t ldo, hipStream_t st);
// r_u = Re x, r_l = a Re x - b Im x + v_u from the interleaved complex x.
void launch_cshift_out(int64_t n, int nb, const double* x, int64_t ldx, double a, double b, const double* vu,
                       int64_t ldv, double* ru, double* rl, int64_t ldr, hipStream_t st);
// out = -i in for m interleaved complex values.
void launch_times_minus_i(int64_t m, const double* in, double* out, hipStream_t st);

}  // namespace riga
