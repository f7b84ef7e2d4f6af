// Internal state of one solver handle and the host helpers shared by the
// single-problem and the batched entry points.
#pragma once
#include "../../include/riga.h"

#include <hip/hip_runtime.h>

#include <complex>
#include <functional>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "small_eig.hpp"

namespace riga {
namespace detail {

struct HipError {
  hipError_t e;
};
inline void ck(hipError_t e) {
  if (e != hipSuccess) throw HipError{e};
}

}  // namespace detail
}  // namespace riga

struct riga_problem {
  int device = 0;
  hipStream_t st = nullptr;
  riga_mesh mesh{};
  riga::Plan plan;
  std::vector<void*> allocs;
  riga::DevSpace ds{};
  riga::DevTree dt{};
  int* d_level_nodes = nullptr;
  double *d_gx = nullptr, *d_gw = nullptr, *d_tabM = nullptr, *d_tabK = nullptr;
  double *d_M1 = nullptr, *d_K1 = nullptr;          // banded 1-D factors of M and K (launch_band_1d)
  double *d_K = nullptr, *d_M = nullptr, *d_C = nullptr;
  double* d_A = nullptr;                            // sigma M + C (formed at factor time)
  // Gyroscopic damping (C = alpha M + beta K + G, G skew): element tables and
  // band of int B_i B_j', the values of C^T on C's pattern, and the second
  // triangle of every nonsymmetric front (front, update, factor, inverses).
  // H(curl) space: dense 1-D matrices of the degree-(p-1) space A and the
  // degree-p space B (MA, MB, KB, D = int A_a B_b')
  double *d_hMA = nullptr, *d_hMB = nullptr, *d_hKB = nullptr, *d_hD = nullptr;
  // H(div) space: the degree-p space of y differs from that of x (walls):
  // its MB, KB and D (the x ones above)
  double *d_hMBy = nullptr, *d_hKBy = nullptr, *d_hDy = nullptr;
  bool gyro = false;
  double gx = 0.0, gy = 0.0;
  // Complex target shift sigma + i csig_im (riga_factor_complex; then
  // factored is false and cmode true): the real form of -i Q(sigma) factored
  // on a second handle over the doubled plan, and the operator's scratch
  // (d_cw: M v_u | C v_u + M v_l, N x 4 each; d_cb, d_cx: right-hand sides
  // and solutions of the real form, 2N x 4 each).
  bool cmode = false;
  double csig_im = 0.0;
  riga_problem* cshadow = nullptr;
  double *d_cw = nullptr, *d_cb = nullptr, *d_cx = nullptr;
  // spectrum slicing: [K U_g | M U_g] of the near-degenerate groups (N x 2
  // grp_cols), their Gram blocks and rotations (grp_cols x 16 + 64)
  double *d_grp = nullptr, *d_grpG = nullptr;
  int grp_cols = 0;
  double *d_tabS = nullptr, *d_S1 = nullptr, *d_Ct = nullptr;
  double *d_LR = nullptr, *d_UR = nullptr, *d_TR = nullptr, *d_DR = nullptr;
  double *d_L = nullptr, *d_U = nullptr, *d_T = nullptr, *d_upd = nullptr, *d_tmp = nullptr, *d_tmp2 = nullptr;
  double *d_Lp = nullptr, *d_Tp = nullptr;         // F in the sweep layouts
  int64_t lpsize = 0, tpsize = 0;
  riga::SweepTask *d_ftasks = nullptr, *d_btasks = nullptr;   // solve tasks, grouped by level
  // sliced-ELL copies of sigma M + C and M for the Krylov products
  riga::EllSlab* d_slabs = nullptr;
  int nslab = 0;
  double *d_Aell = nullptr, *d_Mell = nullptr;
  riga::DevSpace* d_space1 = nullptr;   // the problem's space as a one-entry device table
  std::vector<int> node_inst;                     // forest: problem of every node (set before setup)
  double* d_D = nullptr;                            // 64x64 diagonal-block inverses
  std::vector<int> lvl_max_no, lvl_max_nf, lvl_max_cnb, lvl_max_kids;
  std::vector<int> fvar, bvar;                      // sweep tile shape per level (autotuned)
  double* d_tune = nullptr;                         // autotuner output block (ndof x 4)
  std::vector<int> ftask_off, btask_off;
  int64_t* d_status = nullptr;      // [0] first failed pivot (-1: none), [1] negative pivots
  double* d_sgn = nullptr;          // pivot signs of the signed factorization (ndof)
  bool gep = false;                 // the factor is K - s M (signed form), not Q(sigma)
  double* d_part = nullptr;       // reduction scratch
  int64_t upd_len = 0;
  bool assembled = false, factored = false;
  double alpha = 0, beta = 0, sigma = 0;
  const double* c_elem = nullptr;
  double norms[3] = {-1, -1, -1};  // ||K||_1, ||C||_1, ||M||_1
  riga_stats_t stats{};
  // Krylov workspace
  int64_t kw_cols = 0, kw_b = 0, kw_nev = 0;
  double *Vu = nullptr, *Vl = nullptr, *Wl = nullptr, *Vu2 = nullptr, *Vl2 = nullptr, *Wl2 = nullptr;
  double *Ru = nullptr, *Rl = nullptr, *MRl = nullptr, *Tv = nullptr;
  double *d_small = nullptr;      // device staging for h1, h2, G and small matrices
  double *d_H = nullptr;          // device copy of the projected matrix (fast path)
  int* d_flag = nullptr;          // breakdown flag of the fast path
  double *P = nullptr, *MP = nullptr, *CP = nullptr, *KP = nullptr;
  // Compact (TOAR) Krylov workspace: U and its restart copy (N x cols), the
  // operator input [v_u | v_l] (N x 2b) and M v_l, the operator's output, the
  // compact basis [Q1; Q2] (2 x cols x cols), the coordinates of the
  // orthonormalised upper block (cols x 4), the packed next block (cols x 8),
  // small device scratch, the projected matrix and the breakdown flag.
  int64_t tw_cols = 0, tw_b = 0;
  double *tU = nullptr, *tU2 = nullptr, *tX = nullptr, *tW = nullptr, *tRu = nullptr, *tRl = nullptr, *tTv = nullptr;
  double *tQ = nullptr, *tS = nullptr, *tP = nullptr, *tsmall = nullptr, *tH = nullptr;
  int* tflag = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // The Krylov loop runs on a stream of its own (fenced to the caller's stream)
  // so that its block steps can be captured as HIP graphs and replayed.
  hipStream_t own_st = nullptr;
  hipEvent_t ev_fence = nullptr;
  double* pin = nullptr;            // pinned host staging (projected matrix, small blocks)
  size_t pin_len = 0;
  double* pinned(size_t len) {
    if (pin_len < len) {
      if (pin) hipHostFree(pin);
      pin = nullptr;
      pin_len = 0;
      if (hipHostMalloc((void**)&pin, len * sizeof(double), 0) != hipSuccess) throw std::bad_alloc();
      pin_len = len;
    }
    return pin;
  }
  // (k, b, V_u, operator already applied, leading dimension of H): captured
  // block steps.  They bake in the operator's coefficients (sigma, alpha,
  // beta, the damping branch) and the factor, so assembling or factoring
  // again drops them.
  std::map<std::tuple<int, int, const double*, int, int>, hipGraphExec_t> graphs;
  double graph_sigma = 0.0;
  int64_t graph_key = 0;            // factor mode the captured graphs were recorded for
  // Mixed-precision factor: nodes of height < mixed_thr are FP32 (same offsets
  // as the FP64 blocks, in arrays of their own); every solve is refined
  // ir_sweeps times with FP64 residuals of Q, whose values are kept in d_Q.
  bool mixed = false;
  int mixed_thr = 0, ir_sweeps = 0;
  float *d_L32 = nullptr, *d_T32 = nullptr, *d_U32 = nullptr, *d_D32 = nullptr;
  float *d_Lp32 = nullptr, *d_Tp32 = nullptr;
  double *d_Q = nullptr, *d_irX = nullptr, *d_irR = nullptr, *d_irD = nullptr;
  unsigned char* d_prec = nullptr;
  int prec_thr = -1;                // threshold d_prec was written for
  int64_t n_ir = 0;                 // refinement sweeps issued outside the Krylov loop
  double solve_bytes_now = 0.0;     // factor bytes one sweep pass reads (current precision)
  int64_t factor_key() const { return mixed ? 1 + (int64_t)ir_sweeps * 64 + (int64_t)mixed_thr * 4096 : 0; }
  bool level_f32(int lv) const { return mixed && lv < mixed_thr; }

  void clear_graphs() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
  }

  template <class T>
  T* dalloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    allocs.push_back(p);
    return (T*)p;
  }
  void dfree(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) { hipFree(p); allocs.erase(it); }
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* d = dalloc<T>(v.size());
    if (!v.empty()) riga::detail::ck(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
  }
  int64_t N() const { return plan.ndof; }
};

namespace riga {
struct KsCycle;
namespace detail {

// A returned eigenpair counts as converged when its scaled residual (Tisseur's
// backward error of the QEP, 1-norms of K, C, M) is at most this.
constexpr double kEtaConverged = 1e-10;
// Mixed factor, refinement to the floor (ir_tol = 0): the calibration solve
// must bring ||b - Q x|| / ||b|| to at most this before a sweep gains less
// than a factor 4, else the refinement has stagnated.
constexpr double kIrStagnation = 1e-10;

// Maps the library's exceptions to status codes.
riga_status run(const std::function<riga_status()>& f);
// (p+1)-point Gauss--Legendre rule on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Canonical order: increasing |lam - sigma|, clusters by decreasing Im, then Re.
std::vector<int> canonical_order(const std::vector<cplx>& lam, double sigma);
// The plan of a mesh (scalar, curl- or divergence-conforming space); 0 on success.
int build_plan(riga::Plan& P, const riga_mesh& m);
// Upload h->plan and allocate every device array of the handle.
void setup_device(riga_problem* h);
// Sliced-ELL slabs over the row ranges {problem, first row, end row} and the
// two ELL value arrays.
void setup_ell(riga_problem* h, const std::vector<int4>& ranges);
// Device workspace of a solve: the forward sweep's result (tmp, ndof x nrhs),
// the update vectors passed up the tree (upd, upd_len x nrhs) and, for a mixed
// factor, the refinement's iterate, residual and correction (ndof x nrhs
// each).  Every entry a solve reads from it was written earlier in the same
// solve, so the contents between solves do not matter.
struct SolveWork {
  double *tmp, *upd, *irX, *irR, *irD;
};
// The handle's own workspace (allocated with the handle and the mixed factor).
SolveWork handle_work(const riga_problem* h);
// Solves with the factor (see api.cpp); w = nullptr takes the handle's workspace.
void sweep(riga_problem* h, int nrhs, const double* b, int64_t ldb, const riga::BwdOut& o,
           const SolveWork* w = nullptr);
void solve_levels(riga_problem* h, int nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                  double* r_l, const double* v_u, int64_t ldv, double sig, const SolveWork* w = nullptr);
void factor_level(riga_problem* h, int lv, double s2, double s1);
// Factor every level; RIGA_ERR_NOT_SPD with *bad_pivot (a dof) on a failed pivot.
riga_status factor_all(riga_problem* h, double sigma, int64_t* bad_pivot);
// K - shift M in the signed form L S L^T; *negs = negative pivots (the number
// of eigenvalues of K u = mu M u below shift).
riga_status factor_gep_all(riga_problem* h, double shift, int64_t* bad_pivot, int64_t* negs);
void ensure_norms(riga_problem* h);
void ensure_krylov(riga_problem* h, int cols, int b);
void ensure_post(riga_problem* h, int nev);
// S v for a block of nb vectors (eq. BlockOperatorVector) with M v_l supplied:
// ru = -Q(sigma)^{-1} ((sigma M + C) vu + wl), rl = sigma ru + vu; t: N x nb scratch.
void apply_block(riga_problem* h, int nb, const double* vu, const double* wl, int64_t ld,
                 double* ru, double* rl, double* t);
// Eigenpairs from the planar Ritz vectors of cyc's wanted values in h->P (see api.cpp).
int finish_pairs(riga_problem* h, const riga::KsCycle& cyc, int nev, double* dsmall, double* lam, double* X,
                 double* eta);
// The nev eigenpairs nearest sigma by block Krylov--Schur with the compact
// (TOAR) basis (see toar.cpp).  Sets *fallback (and returns RIGA_OK, nothing
// written) when the compact form cannot run the case; the caller then runs
// the full-basis iteration.
riga_status eigs_toar(riga_problem* h, const riga_options* opt, int nev, int b, int m, int maxit, double tol,
                      double* lam, double* X, double* eta, int* nconv, bool* fallback);
int small_chol(int b, const std::vector<double>& G, std::vector<double>& R, double rel);
// Dense 1-D matrices of the H(curl) space (see hcurl.cpp).
void hcurl_1d(const riga::Space1D& A, const riga::Space1D& B, std::vector<double>& MA, std::vector<double>& MB,
              std::vector<double>& KB, std::vector<double>& D);
// M X for nq columns (ld N): the sum-factorised product on the scalar space,
// the sparse product with explicit columns on a vector space.
void mass_product(riga_problem* h, int nq, const double* X, double* Y);
// Autotune the per-level sweep shapes of a factored handle (see riga_autotune).
void autotune_sweeps(riga_problem* h, int nrhs, int reps, double* before_ms, double* after_ms);
std::vector<double> upper_inverse(int b, const std::vector<double>& R);

}  // namespace detail
}  // namespace riga
