// C ABI of the solver and the host driver of the Krylov iteration.
//
// Everything that touches N-sized data runs in the device kernels; the host
// keeps only the projected matrix (at most ~100 x 100) and the tree plan.
#include "problem.hpp"
#include "ks_host.hpp"
#include "sweep_plan.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>

using riga::cplx;
using namespace riga::detail;

namespace riga {
namespace detail {

// (p+1)-point Gauss--Legendre rule on [-1, 1]: Newton iteration on the
// three-term Legendre recurrence started from the Chebyshev-like guesses.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      double dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::abs(dz) < 1e-16) {
        // final derivative at the converged node
        p0 = 1.0; p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        break;
      }
    }
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
      double p2 = p1;
      p1 = p0;
      p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    double dp = n * (z * p0 - p1) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Canonical order of eigenvalues: increasing |lam - sigma|, clusters (relative
// 1e-9) by decreasing Im, then increasing Re.
std::vector<int> canonical_order(const std::vector<cplx>& lam, double sigma) {
  std::vector<int> idx(lam.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    return std::abs(lam[a] - sigma) < std::abs(lam[b] - sigma);
  });
  std::vector<int> out;
  size_t i = 0;
  while (i < idx.size()) {
    double d0 = std::abs(lam[idx[i]] - sigma);
    size_t j = i + 1;
    while (j < idx.size() && std::abs(lam[idx[j]] - sigma) - d0 <= 1e-9 * std::max(d0, 1e-300)) ++j;
    std::vector<int> g(idx.begin() + i, idx.begin() + j);
    std::stable_sort(g.begin(), g.end(), [&](int a, int b) {
      if (lam[a].imag() != lam[b].imag()) return lam[a].imag() > lam[b].imag();
      return lam[a].real() < lam[b].real();
    });
    out.insert(out.end(), g.begin(), g.end());
    i = j;
  }
  return out;
}

}  // namespace detail
}  // namespace riga


namespace riga {
namespace detail {

riga_status run(const std::function<riga_status()>& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return RIGA_ERR_OOM;
  } catch (const HipError&) {
    return RIGA_ERR_HIP;
  }
}

// ---- forward / backward solve -------------------------------------------------
// One forward and one backward sweep over all levels, each level with the
// precision its factor blocks were computed in.
SolveWork handle_work(const riga_problem* h) {
  return SolveWork{h->d_tmp, h->d_upd, h->d_irX, h->d_irR, h->d_irD};
}

void sweep(riga_problem* h, int nrhs, const double* b, int64_t ldb, const riga::BwdOut& o, const SolveWork* w) {
  const SolveWork hw = handle_work(h);
  if (w == nullptr) w = &hw;
  const riga::Plan& P = h->plan;
  const int H = P.height;
  for (int lv = 0; lv < H; ++lv) {
    int a = h->ftask_off[lv], c = h->ftask_off[lv + 1] - a;
    const bool f32 = h->level_f32(lv);
    riga::launch_fwd_level(h->dt, h->d_ftasks + a, c, nrhs, h->d_Lp, f32 ? h->d_Lp32 : nullptr, b, ldb, w->tmp,
                           h->N(), w->upd, h->lvl_max_nf[lv], h->fvar[lv], h->st);
  }
  for (int lv = H - 1; lv >= 0; --lv) {
    int a = h->btask_off[lv], c = h->btask_off[lv + 1] - a;
    const bool f32 = h->level_f32(lv);
    riga::launch_bwd_level(h->dt, h->d_btasks + a, c, nrhs, h->d_Tp, f32 ? h->d_Tp32 : nullptr, w->tmp, h->N(), o,
                           h->lvl_max_nf[lv], h->bvar[lv], h->st);
  }
}

// x = Q^{-1} b, or with r_l the operator epilogue r_u = -Q^{-1} b (into x),
// r_l = sig r_u + v_u.  With the mixed factor the solution is refined with
// FP64 residuals: x_0 = Q~^{-1} b, x_k = x_{k-1} + Q~^{-1}(b - Q x_{k-1}).
// b is read for the last time before x or r_l is written, so either may alias it.
void solve_levels(riga_problem* h, int nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                  double* r_l, const double* v_u, int64_t ldv, double sig, const SolveWork* w) {
  const SolveWork hw = handle_work(h);
  if (w == nullptr) w = &hw;
  const int K = h->mixed ? h->ir_sweeps : 0;
  riga::BwdOut o;
  if (K == 0) {
    o.xs = x; o.ldxs = ldx; o.neg = r_l != nullptr ? 1 : 0;
    o.rl = r_l; o.v_u = v_u; o.ldv = ldv; o.ldr = ldx; o.sig = sig;
    sweep(h, nrhs, b, ldb, o, w);
    return;
  }
  const int64_t N = h->N();
  o.xs = w->irX; o.ldxs = N;
  sweep(h, nrhs, b, ldb, o, w);
  for (int k = 1; k <= K; ++k) {
    riga::launch_spmv(h->ds, N, nrhs, h->d_Q, -1.0, w->irX, N, w->irR, N, b, ldb,
                      1.0, nullptr, 0, h->st);
    riga::BwdOut c;
    c.xs = w->irD; c.ldxs = N;
    c.base = w->irX; c.ldbase = N;
    if (k < K) {
      c.ru = w->irX; c.ldr = N;
    } else {
      c.ru = x; c.ldr = ldx;
      c.scale = r_l != nullptr ? -1.0 : 1.0;
      c.rl = r_l; c.v_u = v_u; c.ldv = ldv; c.sig = sig;
    }
    sweep(h, nrhs, w->irR, N, c, w);
  }
}

// S v for a block of `nb` vectors (eq. BlockOperatorVector):
//   t = (sigma M + C) v_u + (M v_l),   r_u = -Q^{-1} t,   r_l = sigma r_u + v_u,
// with M v_l supplied (Wl) and sigma M + C formed at factor time.
void apply_block(riga_problem* h, int nb, const double* vu, const double* wl, int64_t ld,
                 double* ru, double* rl, double* t) {
  const int64_t N = h->N();
  if (h->cmode) {
    // the real part of the operator at sigma = a + ib: t = (a M + C) v_u + M v_l
    // + i b M v_u, x = -Q(sigma)^{-1} t by the real form on the second
    // handle (same stream), r_u = Re x, r_l = Re(sigma x) + v_u
    riga_problem* sh = h->cshadow;
    sh->st = h->st;
    double* MX = h->d_cw;
    double* CW = h->d_cw + (size_t)4 * N;
    riga::launch_spmv(h->ds, N, nb, h->d_M, 1.0, vu, ld, MX, N, nullptr, 0, 0.0, nullptr, 0, h->st);
    riga::launch_spmv(h->ds, N, nb, h->d_C, 1.0, vu, ld, CW, N, wl, ld, 1.0, nullptr, 0, h->st);
    riga::launch_cshift_rhs(N, nb, MX, CW, N, h->sigma, h->csig_im, h->d_cb, 2 * N, h->st);
    solve_levels(sh, nb, h->d_cb, 2 * N, h->d_cx, 2 * N, nullptr, nullptr, 0, 0.0);
    riga::launch_cshift_out(N, nb, h->d_cx, 2 * N, h->sigma, h->csig_im, vu, ld, ru, rl, N, h->st);
    return;
  }
  if (h->c_elem == nullptr && !h->gyro)   // sigma M + C = (sigma + alpha) M + beta K: sum factorisation
    riga::launch_tensor_mk(h->ds, h->d_M1, h->d_K1, nb, h->sigma + h->alpha, h->beta, vu, ld, t, N, wl, ld, 1.0,
                           h->st);
  else
    riga::launch_spmv_ell(h->d_slabs, h->nslab, h->d_space1, nullptr, nullptr, nb, h->d_Aell, vu, ld, t, N, wl, ld,
                          1.0, h->st);
  solve_levels(h, nb, t, N, ru, N, rl, vu, ld, h->sigma);
}

void mass_product(riga_problem* h, int nq, const double* X, double* Y) {
  const int64_t N = h->N();
  if (h->plan.kind == riga::SPACE_H1)
    riga::launch_tensor_mk(h->ds, h->d_M1, h->d_K1, nq, 1.0, 0.0, X, N, Y, N, nullptr, 0, 0.0, h->st);
  else
    riga::launch_spmv(h->ds, N, nq, h->d_M, 1.0, X, N, Y, N, nullptr, 0, 0.0, nullptr, 0, h->st);
}

// ||K||_1, ||C||_1, ||M||_1 (largest absolute column sums): one launch, one copy.
void ensure_norms(riga_problem* h) {
  if (h->norms[0] >= 0) return;
  const int rows = 1024;
  const int nblk = (int)((h->N() + rows - 1) / rows);
  double* part = h->d_part;   // 512 * 400 * 4 doubles: room for 3 per block up to 280M rows
  // largest absolute column sums: the row sums of the symmetric K and M, and
  // of C^T when the damping has a skew part
  riga::launch_rowabs3(nullptr, nblk, h->N(), rows, h->ds.rowptr, h->d_K, h->gyro ? h->d_Ct : h->d_C, h->d_M, part,
                       h->st);
  std::vector<double> hp((size_t)nblk * 3);
  ck(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
  ck(hipStreamSynchronize(h->st));
  for (int a = 0; a < 3; ++a) {
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = std::max(m, hp[(size_t)b * 3 + a]);
    h->norms[a] = m;
  }
}

void ensure_krylov(riga_problem* h, int cols, int b) {
  if (h->kw_cols >= cols && h->kw_b >= b) return;
  h->clear_graphs();
  for (double* p : {h->Vu, h->Vl, h->Wl, h->Vu2, h->Vl2, h->Wl2, h->Ru, h->Rl, h->MRl, h->Tv,
                    h->d_small, h->d_H})
    h->dfree(p);
  const int64_t N = h->N();
  cols = std::max<int>(cols, (int)h->kw_cols);
  b = std::max<int>(b, (int)h->kw_b);
  h->Vu = h->dalloc<double>(N * cols); h->Vl = h->dalloc<double>(N * cols); h->Wl = h->dalloc<double>(N * cols);
  h->Vu2 = h->dalloc<double>(N * cols); h->Vl2 = h->dalloc<double>(N * cols); h->Wl2 = h->dalloc<double>(N * cols);
  h->Ru = h->dalloc<double>(N * b); h->Rl = h->dalloc<double>(N * b); h->MRl = h->dalloc<double>(N * b);
  h->Tv = h->dalloc<double>(N * b);
  h->d_small = h->dalloc<double>((size_t)4 * cols * cols + 64);
  h->d_H = h->dalloc<double>((size_t)cols * cols);
  if (!h->d_flag) h->d_flag = h->dalloc<int>(4);
  h->kw_cols = cols; h->kw_b = b;
}

void ensure_post(riga_problem* h, int nev) {
  if (h->kw_nev >= nev) return;
  for (double* p : {h->P, h->MP, h->CP, h->KP}) h->dfree(p);
  const int64_t N = h->N();
  h->P = h->dalloc<double>(N * 2 * nev); h->MP = h->dalloc<double>(N * 2 * nev);
  h->CP = h->dalloc<double>(N * 2 * nev); h->KP = h->dalloc<double>(N * 2 * nev);
  h->kw_nev = nev;
}

// Cholesky of a small SPD b x b matrix G = R^T R (R upper, column-major).
// Returns the index of the first failing pivot, or -1.
int small_chol(int b, const std::vector<double>& G, std::vector<double>& R, double rel) {
  R.assign((size_t)b * b, 0.0);
  for (int j = 0; j < b; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = G[i + (size_t)j * b];
      for (int k = 0; k < i; ++k) s -= R[k + (size_t)i * b] * R[k + (size_t)j * b];
      if (i == j) {
        if (!(s > rel * G[j + (size_t)j * b]) || !(s > 0)) return j;
        R[j + (size_t)j * b] = std::sqrt(s);
      } else {
        R[i + (size_t)j * b] = s / R[i + (size_t)i * b];
      }
    }
  }
  return -1;
}

std::vector<double> upper_inverse(int b, const std::vector<double>& R) {
  std::vector<double> X((size_t)b * b, 0.0);
  for (int j = 0; j < b; ++j) {
    X[j + (size_t)j * b] = 1.0 / R[j + (size_t)j * b];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i + (size_t)k * b] * X[k + (size_t)j * b];
      X[i + (size_t)j * b] = -s / R[i + (size_t)i * b];
    }
  }
  return X;
}

void setup_ell(riga_problem* h, const std::vector<int4>& ranges) {
  std::vector<riga::EllSlab> slabs;
  const int64_t entries = riga::build_ell_slabs(h->plan.rowptr, ranges, slabs);
  h->nslab = (int)slabs.size();
  h->d_slabs = h->upload(slabs);
  h->d_Aell = h->dalloc<double>(entries);
  h->d_Mell = h->dalloc<double>(entries);
  h->d_space1 = h->upload(std::vector<riga::DevSpace>{h->ds});
}

// The plan of a mesh: the scalar space, the curl-conforming or the
// divergence-conforming one (riga_mesh.space); 0 on success.
int build_plan(riga::Plan& P, const riga_mesh& m) {
  switch (m.space) {
    case RIGA_SPACE_H1: return m.walls == 0 ? P.build(m.p, m.ne, m.hyper_every, m.leaf) : -1;
    case RIGA_SPACE_HCURL:
    case RIGA_SPACE_HCURL_FREE:
      return m.walls == 0 ? P.build_hcurl(m.p, m.ne, m.hyper_every, m.leaf, m.space == RIGA_SPACE_HCURL) : -1;
    case RIGA_SPACE_HDIV: return P.build_hdiv(m.p, m.ne, m.hyper_every, m.leaf, m.walls);
    default: return -1;
  }
}

void setup_device(riga_problem* h) {
    const riga::Plan& P = h->plan;
    const riga::Space1D& S = P.sp;
    h->ds.p = S.p; h->ds.ne = S.ne; h->ds.n = S.n;
    h->ds.knots = h->upload(S.knots);
    h->ds.sup0 = h->upload(S.sup0); h->ds.sup1 = h->upload(S.sup1);
    h->ds.lo = h->upload(S.lo); h->ds.hi = h->upload(S.hi);
    h->ds.first = h->upload(S.first);
    h->ds.rowptr = h->upload(P.rowptr);
    h->ds.col = nullptr;
    if (P.kind != riga::SPACE_H1) {
      h->ds.col = h->upload(P.col);
      if (P.kind == riga::SPACE_HCURL || P.kind == riga::SPACE_HCURL_FREE) {
        std::vector<double> MA, MB, KB, D;
        hcurl_1d(P.cx[0], P.cy[0], MA, MB, KB, D);   // A = S^{p-1} (x of component 0), B = S^p
        h->d_hMA = h->upload(MA); h->d_hMB = h->upload(MB); h->d_hKB = h->upload(KB); h->d_hD = h->upload(D);
      } else if (P.kind == riga::SPACE_HDIV) {
        // A = S^{p-1} (y of component 0); B = S^p of x (component 0) and of y (component 1)
        std::vector<double> MA, MB, KB, D;
        hcurl_1d(P.cy[0], P.cx[0], MA, MB, KB, D);
        h->d_hMA = h->upload(MA); h->d_hMB = h->upload(MB); h->d_hKB = h->upload(KB); h->d_hD = h->upload(D);
        hcurl_1d(P.cx[1], P.cy[1], MA, MB, KB, D);
        h->d_hMBy = h->upload(MB); h->d_hKBy = h->upload(KB); h->d_hDy = h->upload(D);
      }
    }
    h->dt.nf = h->upload(P.nf); h->dt.no = h->upload(P.no); h->dt.nb = h->upload(P.nb);
    h->dt.loff = h->upload(P.loff); h->dt.uoff = h->upload(P.uoff);
    h->dt.foff = h->upload(P.foff); h->dt.fdofs = h->upload(P.fdofs);
    h->dt.fkey = h->upload(P.fkey); h->dt.fpos = h->upload(P.fpos);
    h->dt.coff = h->upload(P.coff); h->dt.clist = h->upload(P.clist);
    h->dt.moff = h->upload(P.moff); h->dt.maps = h->upload(P.maps);
    riga::SweepPlan sw;
    riga::build_sweep_plan(P, h->node_inst, sw);
    h->upd_len = sw.voff.back();
    h->dt.voff = h->upload(sw.voff);
    h->dt.gptr = h->upload(sw.gptr);
    h->dt.gidx = h->upload(sw.gidx);
    h->dt.gsrc = h->upload(sw.gsrc);
    h->d_level_nodes = h->upload(P.level_nodes);
    std::vector<double> gx, gw;
    gauss_legendre(S.p + 1, gx, gw);
    h->d_gx = h->upload(gx); h->d_gw = h->upload(gw);
    const int np = S.p + 1;
    h->d_tabM = h->dalloc<double>((size_t)S.ne * np * np);
    h->d_tabK = h->dalloc<double>((size_t)S.ne * np * np);
    h->d_M1 = h->dalloc<double>((size_t)S.n * (2 * S.p + 1));
    h->d_K1 = h->dalloc<double>((size_t)S.n * (2 * S.p + 1));
    h->d_tabS = h->dalloc<double>((size_t)S.ne * np * np);
    h->d_S1 = h->dalloc<double>((size_t)S.n * (2 * S.p + 1));
    h->d_K = h->dalloc<double>(P.nnz); h->d_M = h->dalloc<double>(P.nnz); h->d_C = h->dalloc<double>(P.nnz);
    h->d_A = h->dalloc<double>(P.nnz);
    h->d_L = h->dalloc<double>(P.lsize); h->d_U = h->dalloc<double>(P.usize);
    h->d_T = h->dalloc<double>(P.lsize);
    h->lpsize = sw.lpsize;
    h->tpsize = sw.tpsize;
    h->dt.lpoff = h->upload(sw.lpoff);
    h->dt.tpoff = h->upload(sw.tpoff);
    h->dt.ttri = h->upload(sw.ttri);
    h->d_Lp = h->dalloc<double>(h->lpsize);
    h->d_Tp = h->dalloc<double>(h->tpsize);
    {
      std::vector<int64_t> doff(P.nf.size() + 1, 0);
      for (size_t v = 0; v < P.nf.size(); ++v) doff[v + 1] = doff[v] + (P.no[v] + 63) / 64;
      h->dt.doff = h->upload(doff);
      h->d_D = h->dalloc<double>((size_t)doff.back() * 4096);
      h->lvl_max_no.assign(P.height, 0);
      h->lvl_max_nf.assign(P.height, 0);
      h->lvl_max_cnb.assign(P.height, 0);
      h->lvl_max_kids.assign(P.height, 0);
      for (int lv = 0; lv < P.height; ++lv)
        for (int k = P.level_off[lv]; k < P.level_off[lv + 1]; ++k) {
          const int v = P.level_nodes[k];
          h->lvl_max_no[lv] = std::max(h->lvl_max_no[lv], P.no[v]);
          h->lvl_max_nf[lv] = std::max(h->lvl_max_nf[lv], P.nf[v]);
          for (int c : P.nodes[v].children) h->lvl_max_cnb[lv] = std::max(h->lvl_max_cnb[lv], P.nb[c]);
          h->lvl_max_kids[lv] = std::max(h->lvl_max_kids[lv], (int)P.nodes[v].children.size());
        }
    }
    h->ftask_off = sw.ftask_off;
    h->btask_off = sw.btask_off;
    h->fvar = sw.fvar;
    h->bvar = sw.bvar;
    h->d_ftasks = h->upload(sw.ftasks);
    h->d_btasks = h->upload(sw.btasks);
    h->d_upd = h->dalloc<double>((size_t)h->upd_len * 4);
    h->d_tmp = h->dalloc<double>((size_t)P.ndof * 4);
    h->d_tmp2 = h->dalloc<double>((size_t)P.ndof * 4);
    h->d_status = h->dalloc<int64_t>(2);
    h->d_part = h->dalloc<double>((size_t)512 * 400 * 4 + 64);
    ck(hipEventCreate(&h->ev0));
    ck(hipEventCreate(&h->ev1));
    ck(hipEventCreateWithFlags(&h->ev_fence, hipEventDisableTiming));
    ck(hipStreamCreateWithFlags(&h->own_st, hipStreamNonBlocking));
}


// psi(lam) = (1/(lam - sigma) + 1/(lam - conj sigma)) / 2 for sigma = a + ib:
// the eigenvalue of the real part of the shift-and-invert operator.
cplx cshift_psi(cplx lam, double a, double b) {
  const cplx w = lam - a;
  return w / (w * w + b * b);
}

// Order by decreasing |psi|; values whose |psi| agree to 1e-9 relative form a
// cluster (a conjugate pair), ordered by decreasing Im, then increasing Re.
std::vector<int> psi_order(const std::vector<cplx>& lam, double a, double b) {
  std::vector<double> g(lam.size());
  for (size_t k = 0; k < lam.size(); ++k) g[k] = std::abs(cshift_psi(lam[k], a, b));
  std::vector<int> idx(lam.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return g[x] > g[y]; });
  std::vector<int> out;
  size_t i = 0;
  while (i < idx.size()) {
    const double g0 = g[idx[i]];
    size_t j = i + 1;
    while (j < idx.size() && g0 - g[idx[j]] <= 1e-9 * g0) ++j;
    std::vector<int> grp(idx.begin() + i, idx.begin() + j);
    std::stable_sort(grp.begin(), grp.end(), [&](int x, int y) {
      if (lam[x].imag() != lam[y].imag()) return lam[x].imag() > lam[y].imag();
      return lam[x].real() < lam[y].real();
    });
    out.insert(out.end(), grp.begin(), grp.end());
    i = j;
  }
  return out;
}

// The eigenvalue of a Ritz pair of the real part of the operator: of the two
// roots of u^T Q(lam) u = 0 the one whose psi is nearest the Ritz value (the
// other is, for a mode of the symmetric pencil, the conjugate, whose psi is
// the conjugate Ritz value).
cplx cshift_polish(const PairForms& pf, cplx theta, double a, double b) {
  const cplx disc = std::sqrt(pf.qc * pf.qc - 4.0 * pf.qm * pf.qk);
  const cplx r1 = (-pf.qc + disc) / (2.0 * pf.qm), r2 = (-pf.qc - disc) / (2.0 * pf.qm);
  const bool ok1 = std::isfinite(r1.real()) && std::isfinite(r1.imag());
  const bool ok2 = std::isfinite(r2.real()) && std::isfinite(r2.imag());
  if (!ok1 && !ok2) {
    // no quadratic: invert psi on the branch |lam - a| >= b
    const cplx sq = std::sqrt(1.0 - 4.0 * theta * theta * b * b);
    return a + (1.0 + sq) / (2.0 * theta);
  }
  if (!ok2) return r1;
  if (!ok1) return r2;
  return std::abs(cshift_psi(r1, a, b) - theta) <= std::abs(cshift_psi(r2, a, b) - theta) ? r1 : r2;
}

}  // namespace detail
}  // namespace riga

extern "C" {

const char* riga_status_str(riga_status s) {
  switch (s) {
    case RIGA_OK: return "ok";
    case RIGA_ERR_INVALID_ARG: return "invalid argument";
    case RIGA_ERR_NOT_SPD: return "Q(sigma) is not positive definite";
    case RIGA_ERR_HIP: return "HIP runtime error";
    case RIGA_ERR_OOM: return "out of device memory";
    case RIGA_ERR_STATE: return "call out of order";
    case RIGA_ERR_SCRATCH: return "the solve needs more workspace than the static scratch array holds (RIGA_NOALLOC_SCRATCH_BYTES)";
    case RIGA_WARN_NOT_CONVERGED: return "not all requested eigenpairs converged";
    case RIGA_WARN_IR_STAGNATED: return "iterative refinement of the mixed factor stagnated; factored in FP64";
  }
  return "unknown status";
}

riga_status riga_create(riga_problem** out, const riga_mesh* mesh, int device, void* hip_stream) {
  if (!out || !mesh) return RIGA_ERR_INVALID_ARG;
  *out = nullptr;
  riga_problem* h = new (std::nothrow) riga_problem();
  if (!h) return RIGA_ERR_OOM;
  h->mesh = *mesh;
  const int built = build_plan(h->plan, *mesh);
  if (built != 0) {
    delete h;
    return RIGA_ERR_INVALID_ARG;
  }
  riga_status rc = run([&]() -> riga_status {
    ck(hipSetDevice(device));
    h->device = device;
    h->st = (hipStream_t)hip_stream;
    setup_device(h);
    if (h->plan.kind == riga::SPACE_H1) setup_ell(h, {int4{0, 0, (int)h->N(), 0}});
    return RIGA_OK;
  });
  if (rc != RIGA_OK) {
    riga_destroy(h);
    return rc;
  }
  *out = h;
  return RIGA_OK;
}

void riga_destroy(riga_problem* h) {
  if (!h) return;
  if (h->cshadow) {
    riga_problem* sh = h->cshadow;
    h->cshadow = nullptr;
    sh->st = nullptr;   // h's stream: h synchronises it below
    riga_destroy(sh);
  }
  hipSetDevice(h->device);
  if (h->st) hipStreamSynchronize(h->st); else hipDeviceSynchronize();
  if (h->own_st) hipStreamSynchronize(h->own_st);
  h->clear_graphs();
  for (void* p : h->allocs) hipFree(p);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  if (h->ev_fence) hipEventDestroy(h->ev_fence);
  if (h->pin) hipHostFree(h->pin);
  if (h->own_st) hipStreamDestroy(h->own_st);
  delete h;
}

riga_status riga_info(const riga_problem* h, riga_info_t* info) {
  if (!h || !info) return RIGA_ERR_INVALID_ARG;
  const riga::Plan& P = h->plan;
  info->n1d = P.n1d;
  info->ndof = P.ndof;
  info->nnz = P.nnz;
  info->nnodes = (int64_t)P.nodes.size();
  info->nleaves = P.level_off.size() > 1 ? P.level_off[1] : 0;
  info->height = P.height;
  info->max_front = P.max_front;
  info->leaf_own = P.max_own;
  info->factor_entries = P.lsize;
  info->factor_flops_dense = P.flops_dense;
  info->solve_bytes = P.solve_bytes;
  const_cast<riga::Plan&>(P).ensure_symbolic();   // cached on the handle
  info->factor_nnz = P.sym_nnz_l;
  info->factor_flops = P.sym_flops;
  info->upd_len = h->upd_len;
  return RIGA_OK;
}

riga_status riga_symbolic(const riga_mesh* mesh, int64_t* ndof, int64_t* order, int64_t* colcount,
                          int64_t* nnz_l, double* flops) {
  if (!mesh) return RIGA_ERR_INVALID_ARG;
  return run([&]() -> riga_status {
    riga::Plan P;
    const int built = build_plan(P, *mesh);
    if (built != 0) return RIGA_ERR_INVALID_ARG;
    if (ndof) *ndof = P.ndof;
    std::vector<int64_t> cc;
    int64_t nz = 0;
    double fl = 0.0;
    P.symbolic(colcount ? &cc : nullptr, nz, fl);
    if (order)
      for (int64_t d = 0; d < P.ndof; ++d) order[P.elim_pos[d]] = d;
    if (colcount) std::copy(cc.begin(), cc.end(), colcount);
    if (nnz_l) *nnz_l = nz;
    if (flops) *flops = fl;
    return RIGA_OK;
  });
}

namespace {

riga_status assemble_impl(riga_problem* h, const riga_damping* damping, double gx, double gy) {
  if (!h || !damping || !std::isfinite(gx) || !std::isfinite(gy)) return RIGA_ERR_INVALID_ARG;
  if ((gx != 0.0 || gy != 0.0) && !h->node_inst.empty()) return RIGA_ERR_INVALID_ARG;
  if (h->plan.kind != riga::SPACE_H1 && (gx != 0.0 || gy != 0.0 || damping->c_elem != nullptr))
    return RIGA_ERR_INVALID_ARG;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    if (h->plan.kind != riga::SPACE_H1) {
      const riga::Plan& P = h->plan;
      ck(hipEventRecord(h->ev0, h->st));
      if (P.kind == riga::SPACE_HDIV)
        riga::launch_assemble_hdiv(P.cy[0].n, P.cx[0].n, P.cy[1].n, P.cbase[1], P.ndof, h->ds.rowptr, h->ds.col,
                                   h->d_hMA, h->d_hMB, h->d_hKB, h->d_hD, h->d_hMBy, h->d_hKBy, h->d_hDy, P.walls,
                                   damping->alpha, damping->beta, h->d_K, h->d_M, h->d_C, h->st);
      else
        riga::launch_assemble_hcurl(P.cx[0].n, P.cx[1].n, P.cbase[1], P.ndof, h->ds.rowptr, h->ds.col, h->d_hMA,
                                    h->d_hMB, h->d_hKB, h->d_hD, damping->alpha, damping->beta, h->d_K, h->d_M,
                                    h->d_C, h->st);
      ck(hipGetLastError());
      ck(hipEventRecord(h->ev1, h->st));
      h->gyro = false; h->gx = h->gy = 0.0;
      h->alpha = damping->alpha; h->beta = damping->beta; h->c_elem = nullptr;
      h->clear_graphs();
      h->assembled = true;
      h->factored = false;
      h->cmode = false;
      h->norms[0] = h->norms[1] = h->norms[2] = -1;
      h->stats.flops[RIGA_PHASE_ASSEMBLE] = 0.0;
      h->stats.bytes[RIGA_PHASE_ASSEMBLE] = 24.0 * (double)P.nnz;
      h->stats.t_assemble_ms = -1;
      return RIGA_OK;
    }
    const bool gyro = gx != 0.0 || gy != 0.0;
    if (gyro && h->d_Ct == nullptr) {
      const riga::Plan& P = h->plan;
      h->d_Ct = h->dalloc<double>(P.nnz);
      h->d_LR = h->dalloc<double>(P.lsize);
      h->d_UR = h->dalloc<double>(P.usize);
      h->d_TR = h->dalloc<double>(P.lsize);
      int64_t dblocks = 0;
      for (size_t v = 0; v < P.nf.size(); ++v) dblocks += (P.no[v] + 63) / 64;
      h->d_DR = h->dalloc<double>((size_t)dblocks * 4096);
    }
    // captured block steps hold the operator's coefficients (alpha, beta, the
    // skew part) and its kernel choice (an element damping field or not): they
    // are kept only when a re-assembly leaves all of these as they were
    const bool same_op = h->assembled && h->gyro == gyro && h->gx == gx && h->gy == gy &&
                         h->alpha == damping->alpha && h->beta == damping->beta &&
                         (h->c_elem == nullptr) == (damping->c_elem == nullptr);
    if (!same_op) h->clear_graphs();
    ck(hipEventRecord(h->ev0, h->st));
    riga::launch_bspline_tables(h->ds, h->d_gx, h->d_gw, h->d_tabM, h->d_tabK, gyro ? h->d_tabS : nullptr, h->st);
    riga::launch_band_1d(h->ds, h->d_tabM, h->d_tabK, h->d_M1, h->d_K1, h->st);
    if (gyro) riga::launch_band_skew(h->ds, h->d_tabS, h->d_S1, h->st);
    riga::launch_assemble(h->ds, h->d_tabM, h->d_M1, h->d_K1, damping->alpha, damping->beta, damping->c_elem,
                          h->d_K, h->d_M, h->d_C, h->N(), h->st, gyro ? h->d_S1 : nullptr, gx, gy,
                          gyro ? h->d_Ct : nullptr);
    ck(hipGetLastError());
    ck(hipEventRecord(h->ev1, h->st));
    h->gyro = gyro; h->gx = gx; h->gy = gy;
    h->alpha = damping->alpha; h->beta = damping->beta; h->c_elem = damping->c_elem;
    h->assembled = true;
    h->factored = false;
    h->cmode = false;
    // the 1-norms of K, C, M (residual scaling) are those of the same matrices
    // when nothing but an element field's values could have changed, and it is absent
    if (!(same_op && damping->c_elem == nullptr)) h->norms[0] = h->norms[1] = h->norms[2] = -1;
    h->stats.flops[RIGA_PHASE_ASSEMBLE] = 0.0;   // a lower-order term of eq. Cost
    h->stats.bytes[RIGA_PHASE_ASSEMBLE] =
        24.0 * (double)h->plan.nnz + (damping->c_elem ? 8.0 * h->mesh.ne * (double)h->mesh.ne : 0.0);
    h->stats.t_assemble_ms = -1;  // resolved lazily (the call does not synchronise)
    return RIGA_OK;
  });
}

}  // namespace

riga_status riga_assemble(riga_problem* h, const riga_damping* damping) {
  return assemble_impl(h, damping, 0.0, 0.0);
}

riga_status riga_assemble_gyroscopic(riga_problem* h, const riga_damping* damping, double gx, double gy) {
  return assemble_impl(h, damping, gx, gy);
}

riga_status riga_export_csr(riga_problem* h, int which, int64_t* rowptr, int32_t* col, double* val) {
  if (!h || which < 0 || which > 3) return RIGA_ERR_INVALID_ARG;
  if (val && !h->assembled) return RIGA_ERR_STATE;
  if (val && which == 3 && !h->gyro) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    const riga::Plan& P = h->plan;
    const riga::Space1D& S = P.sp;
    if (rowptr) std::memcpy(rowptr, P.rowptr.data(), (P.ndof + 1) * sizeof(int64_t));
    if (col && !P.col.empty()) {
      std::copy(P.col.begin(), P.col.end(), col);
    } else if (col) {
      const int n = S.n;
      int64_t k = 0;
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          for (int jj = S.lo[j]; jj <= S.hi[j]; ++jj)
            for (int ii = S.lo[i]; ii <= S.hi[i]; ++ii) col[k++] = jj * n + ii;
    }
    if (val) {
      const double* src = which == 0 ? h->d_K : which == 1 ? h->d_M : which == 2 ? h->d_C : h->d_Ct;
      ck(hipMemcpyAsync(val, src, P.nnz * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    }
    return RIGA_OK;
  });
}

}  // extern "C"

namespace riga {
namespace detail {

// Factor level lv of the tree (FP32 if the mixed threshold says so): the
// fronts of s2 M + s1 C + K.
void factor_level(riga_problem* h, int lv, double s2, double s1) {
  const riga::Plan& P = h->plan;
  int a = P.level_off[lv], c = P.level_off[lv + 1] - a;
  riga::DevTree t = h->dt;
  if (h->gyro && !h->gep) {   // nonsymmetric Q: LU fronts (FP64)
    riga::launch_front_factor_lu(h->ds, t, h->d_level_nodes + a, c, h->lvl_max_no[lv], h->lvl_max_nf[lv],
                                 h->lvl_max_cnb[lv], h->lvl_max_kids[lv], s2, s1, h->d_K, h->d_M, h->d_C, h->d_Ct,
                                 h->d_L, h->d_U, h->d_T, h->d_D, h->d_LR, h->d_UR, h->d_TR, h->d_DR, h->d_Lp, h->d_Tp,
                                 h->d_status, h->st);
    return;
  }
  if (h->mixed) t.prec = h->d_prec;
  if (h->level_f32(lv))
    riga::launch_front_factor(h->ds, t, h->d_level_nodes + a, c, h->lvl_max_no[lv], h->lvl_max_nf[lv],
                              h->lvl_max_cnb[lv], h->lvl_max_kids[lv], s2, s1, h->d_K, h->d_M, h->d_C, h->d_L32, h->d_U32,
                              h->d_T32, h->d_D32, h->d_Lp32, h->d_Tp32, h->d_status, h->st);
  else
    riga::launch_front_factor(h->ds, t, h->d_level_nodes + a, c, h->lvl_max_no[lv], h->lvl_max_nf[lv],
                              h->lvl_max_cnb[lv], h->lvl_max_kids[lv], s2, s1, h->d_K, h->d_M, h->d_C, h->d_L, h->d_U,
                              h->d_T, h->d_D, h->d_Lp, h->d_Tp, h->d_U32, h->d_status, h->st);
}

// Factor every level; RIGA_ERR_NOT_SPD with *bad_pivot on a failed pivot.
riga_status factor_all(riga_problem* h, double sigma, int64_t* bad_pivot) {
  const riga::Plan& P = h->plan;
  h->dt.sgn = nullptr;
  h->gep = false;
  h->cmode = false;
  ck(hipMemsetAsync(h->d_status, 0xFF, sizeof(int64_t), h->st));
  ck(hipEventRecord(h->ev0, h->st));
  for (int lv = 0; lv < P.height; ++lv) factor_level(h, lv, sigma * sigma, sigma);
  // sigma M + C for the operator, Q(sigma) for the residuals of the mixed factor
  riga::launch_combine3(P.nnz, sigma, h->d_M, 1.0, h->d_C, 0.0, h->d_K, h->d_A, h->st);
  // (a forest combines its per-problem shifts itself and converts then; without
  // an element damping field the operator uses the sum-factorised product)
  if (h->node_inst.empty() && (h->c_elem != nullptr || h->gyro))
    riga::launch_csr_to_ell(h->d_slabs, h->nslab, h->ds.rowptr, h->d_A, h->d_Aell, h->st);
  if (h->mixed) riga::launch_combine3(P.nnz, sigma * sigma, h->d_M, sigma, h->d_C, 1.0, h->d_K, h->d_Q, h->st);
  ck(hipGetLastError());
  ck(hipEventRecord(h->ev1, h->st));
  int64_t stat = -1;
  ck(hipMemcpyAsync(&stat, h->d_status, sizeof(int64_t), hipMemcpyDeviceToHost, h->st));
  ck(hipStreamSynchronize(h->st));
  float ms = 0;
  ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->stats.t_factor_ms = ms;
  {
    riga::Plan& Pm = h->plan;
    // factor entries read by one forward + backward pass, FP32 levels at 4 B
    double sb = 0.0;
    for (size_t v = 0; v < Pm.nodes.size(); ++v) {
      const double o = Pm.no[v], bb = Pm.nb[v];
      sb += 2.0 * (h->level_f32(Pm.nodes[v].height) ? 4.0 : 8.0) * (o * (o + 1) / 2 + bb * o);
    }
    h->solve_bytes_now = sb;
    Pm.ensure_symbolic();
    h->stats.flops[RIGA_PHASE_FACTOR] = Pm.sym_flops;
    h->stats.bytes[RIGA_PHASE_FACTOR] = 24.0 * (double)Pm.nnz + 8.0 * (double)Pm.sym_nnz_l;
  }
  if (stat >= 0) {
    if (bad_pivot) *bad_pivot = stat;
    h->factored = false;
    return RIGA_ERR_NOT_SPD;
  }
  h->sigma = sigma;
  h->factored = true;
  return RIGA_OK;
}

riga_status factor_gep_all(riga_problem* h, double shift, int64_t* bad_pivot, int64_t* negs) {
  const riga::Plan& P = h->plan;
  h->clear_graphs();
  h->mixed = false;
  h->factored = false;
  h->cmode = false;
  if (h->d_sgn == nullptr) h->d_sgn = h->dalloc<double>((size_t)h->N());
  h->dt.sgn = h->d_sgn;
  h->gep = true;
  ck(hipMemsetAsync(h->d_status, 0xFF, sizeof(int64_t), h->st));   // no failed pivot
  ck(hipMemsetAsync(h->d_status + 1, 0, sizeof(int64_t), h->st));   // no negative pivot
  ck(hipEventRecord(h->ev0, h->st));
  for (int lv = 0; lv < P.height; ++lv) factor_level(h, lv, -shift, 0.0);
  ck(hipGetLastError());
  ck(hipEventRecord(h->ev1, h->st));
  int64_t stat[2] = {-1, 0};
  ck(hipMemcpyAsync(stat, h->d_status, sizeof(stat), hipMemcpyDeviceToHost, h->st));
  ck(hipStreamSynchronize(h->st));
  float ms = 0;
  ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->stats.t_factor_ms = ms;
  if (negs) *negs = stat[1];
  if (stat[0] >= 0) {
    if (bad_pivot) *bad_pivot = stat[0];
    return RIGA_ERR_NOT_SPD;
  }
  h->sigma = shift;
  h->factored = true;
  return RIGA_OK;
}

// ||b - Q x|| / ||b|| history of a refined solve of one seeded right-hand side
// (hist[0] after the unrefined solve, hist[k] after k refinement sweeps).
void ir_history(riga_problem* h, int kmax, std::vector<double>& hist) {
  const int64_t N = h->N();
  double* b = h->d_tmp2;
  riga::launch_random_fill(b, N, 1, N, 0x5eed1234ULL, h->st);
  const int nblk = riga::dots_blocks(N);
  double* out = h->d_part + nblk + 8;
  auto norm2 = [&](const double* v) {
    riga::launch_dots(N, 1, v, nullptr, N, 1, v, nullptr, N, h->d_part, out, h->st);
    double r = 0;
    ck(hipMemcpyAsync(&r, out, sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    return std::sqrt(r);
  };
  const double nb = norm2(b);
  riga::BwdOut o;
  o.xs = h->d_irX; o.ldxs = N;
  sweep(h, 1, b, N, o);
  hist.clear();
  for (int k = 0; k <= kmax; ++k) {
    riga::launch_spmv(h->ds, N, 1, h->d_Q, -1.0, h->d_irX, N, h->d_irR, N, b, N, 1.0,
                      nullptr, 0, h->st);
    hist.push_back(norm2(h->d_irR) / nb);
    if (k == kmax) break;
    riga::BwdOut c;
    c.xs = h->d_irD; c.ldxs = N; c.base = h->d_irX; c.ldbase = N; c.ru = h->d_irX; c.ldr = N;
    sweep(h, 1, h->d_irR, N, c);
  }
}

// Per-level autotuning of the sweep shapes.  Every (level, direction) is timed
// with each compiled shape on the handle's own factor and a seeded right-hand
// side, after one full solve has put every level's inputs in place (a level's
// launch only reads what lower / higher levels wrote, so repeating it is
// idempotent).  Choices are cached per device architecture, level structure,
// precision and number of right-hand sides.
void autotune_sweeps(riga_problem* h, int nrhs, int reps, double* before_ms, double* after_ms) {
  static std::mutex mu;
  static std::map<std::string, std::pair<std::vector<int>, std::vector<int>>> cache;
  const riga::Plan& P = h->plan;
  const int H = P.height;
  const int64_t N = h->N();
  hipDeviceProp_t prop;
  ck(hipGetDeviceProperties(&prop, h->device));
  std::string key = std::string(prop.gcnArchName) + "|" + std::to_string(nrhs);
  for (int lv = 0; lv < H; ++lv)
    key += "|" + std::to_string(h->ftask_off[lv + 1] - h->ftask_off[lv]) + "," +
           std::to_string(h->btask_off[lv + 1] - h->btask_off[lv]) + "," + std::to_string(h->lvl_max_nf[lv]) +
           (h->level_f32(lv) ? "s" : "d");
  if (!h->d_tune) h->d_tune = h->dalloc<double>((size_t)N * 4);
  riga::BwdOut o;
  o.xs = h->d_tune; o.ldxs = N;
  auto full = [&]() {
    float ms = 0;
    ck(hipEventRecord(h->ev0, h->st));
    for (int r = 0; r < reps; ++r) sweep(h, nrhs, h->d_tmp2, N, o);
    ck(hipEventRecord(h->ev1, h->st));
    ck(hipEventSynchronize(h->ev1));
    ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    return (double)ms / reps;
  };
  // inputs: a seeded right-hand side (d_tmp2), solved once so that every
  // level's inputs are defined; forward results go to d_tmp, backward to d_tune
  riga::launch_random_fill(h->d_tmp2, N, nrhs, N, 777, h->st);
  sweep(h, nrhs, h->d_tmp2, N, o);
  const double t0 = full();
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      h->fvar = it->second.first;
      h->bvar = it->second.second;
      if (before_ms) *before_ms = t0;
      if (after_ms) *after_ms = full();
      return;
    }
  }
  const int nv = riga::sweep_variants();
  auto time_level = [&](bool fwd, int lv, int var) {
    float ms = 0;
    const bool f32 = h->level_f32(lv);
    ck(hipEventRecord(h->ev0, h->st));
    for (int r = 0; r < reps; ++r) {
      if (fwd) {
        const int a = h->ftask_off[lv], c = h->ftask_off[lv + 1] - a;
        riga::launch_fwd_level(h->dt, h->d_ftasks + a, c, nrhs, h->d_Lp, f32 ? h->d_Lp32 : nullptr, h->d_tmp2, N,
                               h->d_tmp, N, h->d_upd, h->lvl_max_nf[lv], var, h->st);
      } else {
        const int a = h->btask_off[lv], c = h->btask_off[lv + 1] - a;
        riga::launch_bwd_level(h->dt, h->d_btasks + a, c, nrhs, h->d_Tp, f32 ? h->d_Tp32 : nullptr, h->d_tmp, N, o,
                               h->lvl_max_nf[lv], var, h->st);
      }
    }
    ck(hipEventRecord(h->ev1, h->st));
    ck(hipEventSynchronize(h->ev1));
    ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    return (double)ms;
  };
  // forward levels first (they rewrite d_tmp with the same values), then backward
  for (int dir = 0; dir < 2; ++dir)
    for (int lv = 0; lv < H; ++lv) {
      int best = 0;
      double tb = 1e300;
      for (int v = 0; v < nv; ++v) {
        const double t = time_level(dir == 0, lv, v);
        if (t < tb) { tb = t; best = v; }
      }
      (dir == 0 ? h->fvar : h->bvar)[lv] = best;
    }
  {
    std::lock_guard<std::mutex> lock(mu);
    cache[key] = {h->fvar, h->bvar};
  }
  h->clear_graphs();
  if (before_ms) *before_ms = t0;
  if (after_ms) *after_ms = full();
}

}  // namespace detail
}  // namespace riga

extern "C" {

riga_status riga_factor(riga_problem* h, double sigma, int64_t* bad_pivot) {
  if (bad_pivot) *bad_pivot = -1;
  if (!h || !(sigma > 0.0) || !std::isfinite(sigma)) return RIGA_ERR_INVALID_ARG;
  if (!h->assembled) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    // captured block steps stay valid for the same shift and factor kind
    // (riga_eigs compares both before replaying them)
    h->mixed = false;
    return factor_all(h, sigma, bad_pivot);
  });
}

riga_status riga_factor_complex(riga_problem* h, double sigma_re, double sigma_im, int64_t* bad_pivot) {
  if (bad_pivot) *bad_pivot = -1;
  if (!h || !std::isfinite(sigma_re) || !std::isfinite(sigma_im) || !(sigma_im > 0.0)) return RIGA_ERR_INVALID_ARG;
  if (!h->assembled) return RIGA_ERR_STATE;
  if (h->gyro || !h->node_inst.empty()) return RIGA_ERR_INVALID_ARG;   // symmetric damping, one problem
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    h->clear_graphs();
    h->mixed = false;
    h->gep = false;
    h->factored = false;
    h->cmode = false;
    const int64_t N = h->N();
    if (h->cshadow == nullptr) {
      riga_problem* sh = new riga_problem();
      sh->mesh = h->mesh;
      if (sh->plan.build_realform(h->plan) != 0) {
        delete sh;
        return RIGA_ERR_INVALID_ARG;
      }
      h->cshadow = sh;   // owned by h from here (riga_destroy)
      sh->device = h->device;
      sh->st = h->st;
      setup_device(sh);
      const riga::Plan& P = sh->plan;
      sh->gyro = true;   // nonsymmetric: the LU fronts
      sh->d_Ct = sh->dalloc<double>(P.nnz);
      sh->d_LR = sh->dalloc<double>(P.lsize);
      sh->d_UR = sh->dalloc<double>(P.usize);
      sh->d_TR = sh->dalloc<double>(P.lsize);
      int64_t dblocks = 0;
      for (size_t v = 0; v < P.nf.size(); ++v) dblocks += (P.no[v] + 63) / 64;
      sh->d_DR = sh->dalloc<double>((size_t)dblocks * 4096);
      // the real form has no mass term: the fronts read M with coefficient 0
      ck(hipMemsetAsync(sh->d_M, 0, (size_t)P.nnz * sizeof(double), h->st));
      h->d_cw = h->dalloc<double>((size_t)8 * N);
      h->d_cb = h->dalloc<double>((size_t)8 * N);
      h->d_cx = h->dalloc<double>((size_t)8 * N);
    }
    riga_problem* sh = h->cshadow;
    sh->st = h->st;
    const riga::Plan& P = sh->plan;
    ck(hipMemsetAsync(sh->d_status, 0xFF, sizeof(int64_t), h->st));
    ck(hipEventRecord(h->ev0, h->st));
    riga::launch_realform_values(N, h->ds.rowptr, h->d_K, h->d_M, h->d_C, sigma_re, sigma_im, sh->d_K, sh->d_C,
                                 sh->d_Ct, h->st);
    for (int lv = 0; lv < P.height; ++lv) factor_level(sh, lv, 0.0, 1.0);
    ck(hipGetLastError());
    ck(hipEventRecord(h->ev1, h->st));
    int64_t stat = -1;
    ck(hipMemcpyAsync(&stat, sh->d_status, sizeof(int64_t), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    float ms = 0;
    ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->stats.t_factor_ms = ms;
    double sb = 0.0;
    for (size_t v = 0; v < P.nodes.size(); ++v) {
      const double o = P.no[v], bb = P.nb[v];
      sb += 2.0 * 8.0 * (o * (o + 1) / 2 + bb * o);
    }
    h->solve_bytes_now = sb;
    h->stats.flops[RIGA_PHASE_FACTOR] = P.flops_dense * 2.0;   // two triangles
    h->stats.bytes[RIGA_PHASE_FACTOR] = 24.0 * (double)P.nnz + 16.0 * (double)P.lsize;
    if (stat >= 0) {
      if (bad_pivot) *bad_pivot = stat / 2;   // the dof of the failed unknown
      return RIGA_ERR_NOT_SPD;
    }
    h->sigma = sigma_re;
    h->csig_im = sigma_im;
    h->cmode = true;
    h->graph_sigma = std::numeric_limits<double>::quiet_NaN();   // captured steps hold the old shift
    return RIGA_OK;
  });
}

riga_status riga_solve_q_complex(riga_problem* h, int nrhs, const double* b, double* x) {
  if (!h || nrhs < 1 || !b || !x) return RIGA_ERR_INVALID_ARG;
  if (!h->cmode) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    const int64_t N = h->N();
    riga_problem* sh = h->cshadow;
    sh->st = h->st;
    for (int c0 = 0; c0 < nrhs; c0 += 4) {
      const int nc = std::min(4, nrhs - c0);
      riga::launch_times_minus_i(N * nc, b + (size_t)c0 * 2 * N, h->d_cb, h->st);
      solve_levels(sh, nc, h->d_cb, 2 * N, x + (size_t)c0 * 2 * N, 2 * N, nullptr, nullptr, 0, 0.0);
    }
    ck(hipGetLastError());
    return RIGA_OK;
  });
}

riga_status riga_factor_mixed(riga_problem* h, double sigma, int fp64_levels, int ir_sweeps, double ir_tol,
                              double* ir_hist, int64_t* bad_pivot) {
  if (bad_pivot) *bad_pivot = -1;
  if (!h || !(sigma > 0.0) || !std::isfinite(sigma) || fp64_levels < 0 || ir_sweeps < -1 ||
      ir_sweeps > RIGA_IR_MAX || !(ir_tol >= 0.0))
    return RIGA_ERR_INVALID_ARG;
  if (!h->assembled) return RIGA_ERR_STATE;
  if (h->gyro || h->plan.kind != riga::SPACE_H1) return RIGA_ERR_INVALID_ARG;   // FP64 LU / vector space
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    h->clear_graphs();
    const riga::Plan& P = h->plan;
    const int64_t N = h->N();
    if (!h->d_L32) {
      std::vector<int64_t> doff_last(1);
      ck(hipMemcpy(doff_last.data(), h->dt.doff + P.nf.size(), sizeof(int64_t), hipMemcpyDeviceToHost));
      h->d_L32 = h->dalloc<float>(P.lsize); h->d_T32 = h->dalloc<float>(P.lsize);
      h->d_Lp32 = h->dalloc<float>(h->lpsize); h->d_Tp32 = h->dalloc<float>(h->tpsize);
      h->d_U32 = h->dalloc<float>(P.usize);
      h->d_D32 = h->dalloc<float>((size_t)doff_last[0] * 4096);
      h->d_Q = h->dalloc<double>(P.nnz);
      h->d_irX = h->dalloc<double>((size_t)N * 4); h->d_irR = h->dalloc<double>((size_t)N * 4);
      h->d_irD = h->dalloc<double>((size_t)N * 4);
      h->d_prec = h->dalloc<unsigned char>(P.nf.size());
    }
    const int keep = std::min(std::max(fp64_levels, 1), P.height);
    const int thr = P.height - keep;
    if (h->prec_thr != thr) {
      std::vector<unsigned char> prec(P.nf.size(), 0);
      for (size_t v = 0; v < P.nodes.size(); ++v) prec[v] = P.nodes[v].height < thr ? 1 : 0;
      ck(hipMemcpy(h->d_prec, prec.data(), prec.size(), hipMemcpyHostToDevice));
      h->prec_thr = thr;
    }
    h->mixed = true;
    h->mixed_thr = thr;
    h->ir_sweeps = 0;
    riga_status rc = factor_all(h, sigma, bad_pivot);
    if (rc != RIGA_OK) return rc;
    bool stagnated = false;
    if (ir_sweeps < 0 || ir_hist || ir_tol > 0.0) {
      std::vector<double> hist;
      ir_history(h, RIGA_IR_MAX, hist);
      if (ir_hist)
        for (int k = 0; k <= RIGA_IR_MAX; ++k) ir_hist[k] = k < (int)hist.size() ? hist[k] : -1.0;
      if (ir_sweeps < 0) {
        // fewest sweeps reaching ir_tol, and never past the point where a
        // further sweep gains less than a factor 4
        int best = 0;
        for (int k = 1; k < (int)hist.size(); ++k) {
          if (hist[best] <= ir_tol || hist[k] > 0.25 * hist[best]) break;
          best = k;
        }
        ir_sweeps = best;
        // the refinement stopped gaining before the target (ir_tol, or the
        // stagnation bound when refining to the floor)
        const double target = ir_tol > 0.0 ? ir_tol : kIrStagnation;
        stagnated = !(hist[best] <= target);
      } else if (ir_tol > 0.0) {
        // a fixed count must reach the caller's target
        stagnated = !(hist[std::min<int>(ir_sweeps, (int)hist.size() - 1)] <= ir_tol);
      }
    }
    if (stagnated) {
      // the FP32 factor is too weak for the FP64 refinement: factor in FP64
      h->mixed = false;
      h->ir_sweeps = 0;
      rc = factor_all(h, sigma, bad_pivot);
      return rc == RIGA_OK ? RIGA_WARN_IR_STAGNATED : rc;
    }
    h->ir_sweeps = ir_sweeps;
    return RIGA_OK;
  });
}

riga_status riga_autotune(riga_problem* h, int nrhs, int reps, double* before_ms, double* after_ms) {
  if (!h || nrhs < 1 || nrhs > 4 || reps < 1) return RIGA_ERR_INVALID_ARG;
  if (!h->factored) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    autotune_sweeps(h, nrhs, reps, before_ms, after_ms);
    return RIGA_OK;
  });
}

riga_status riga_sweep_shapes(const riga_problem* h, int* fwd, int* bwd, int* levels) {
  if (!h) return RIGA_ERR_INVALID_ARG;
  if (levels) *levels = h->plan.height;
  for (int lv = 0; lv < h->plan.height; ++lv) {
    if (fwd) fwd[lv] = h->fvar[lv];
    if (bwd) bwd[lv] = h->bvar[lv];
  }
  return RIGA_OK;
}

riga_status riga_ir_sweeps(const riga_problem* h, int* sweeps) {
  if (!h || !sweeps) return RIGA_ERR_INVALID_ARG;
  *sweeps = h->mixed ? h->ir_sweeps : -1;
  return RIGA_OK;
}

riga_status riga_solve_q(riga_problem* h, int nrhs, const double* b, double* x) {
  if (!h || nrhs < 1 || nrhs > 4 || !b || !x) return RIGA_ERR_INVALID_ARG;
  if (!h->factored) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    solve_levels(h, nrhs, b, h->N(), x, h->N(), nullptr, nullptr, 0, 0.0);
    ck(hipGetLastError());
    return RIGA_OK;
  });
}

riga_status riga_apply_op(riga_problem* h, int nvec, const double* v, double* r) {
  if (!h || nvec < 1 || nvec > 4 || !v || !r || v == r) return RIGA_ERR_INVALID_ARG;
  if (h->plan.kind != riga::SPACE_H1) return RIGA_ERR_INVALID_ARG;
  if (!h->factored || h->gep) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    const int64_t N = h->N();
    // M v_l into tmp2, then the common block operator
    riga::launch_spmv(h->ds, N, nvec, h->d_M, 1.0, v + N, 2 * N, h->d_tmp2, N,
                      nullptr, 0, 0.0, nullptr, 0, h->st);
    double* t = r + N;  // r_l doubles as scratch for t until the backward sweep writes it
    double* mvu = h->d_upd;  // unused here; Y2 not requested
    (void)mvu;
    riga::launch_spmv(h->ds, N, nvec, h->d_A, 1.0, v, 2 * N, t, 2 * N,
                      h->d_tmp2, N, 1.0, nullptr, 0, h->st);
    solve_levels(h, nvec, t, 2 * N, r, 2 * N, r + N, v, 2 * N, h->sigma);
    ck(hipGetLastError());
    return RIGA_OK;
  });
}

riga_status riga_stats(const riga_problem* h, riga_stats_t* stats) {
  if (!h || !stats) return RIGA_ERR_INVALID_ARG;
  *stats = h->stats;
  return RIGA_OK;
}

riga_status riga_selftest_small_eig(int n, const double* a, double* w, double* resid) {
  if (n < 1 || !a || !w) return RIGA_ERR_INVALID_ARG;
  // the path of the Ritz step: real Schur form, eigenvalues of its blocks,
  // eigenvectors by back-substitution through the quasi-triangular form
  std::vector<double> TR, QR;
  std::vector<cplx> theta, Y;
  if (riga::schur_real(n, a, TR, QR) != 0) return RIGA_WARN_NOT_CONVERGED;
  riga::schur_real_eigvals(n, TR, theta);
  riga::schur_eigvecs_real(n, TR, QR, theta, Y, 1e-12);
  double an = 0.0;
  for (int i = 0; i < n * n; ++i) an = std::max(an, std::abs(a[i]));
  double worst = 0.0;
  for (int k = 0; k < n; ++k) {
    cplx lam = theta[k];
    w[2 * k] = lam.real();
    w[2 * k + 1] = lam.imag();
    for (int i = 0; i < n; ++i) {
      cplx s = 0.0;
      for (int j = 0; j < n; ++j) s += a[i + (size_t)j * n] * Y[j + (size_t)k * n];
      worst = std::max(worst, std::abs(s - lam * Y[i + (size_t)k * n]) / std::max(an, 1e-300));
    }
  }
  if (resid) *resid = worst;
  return RIGA_OK;
}

riga_status riga_selftest_schur_restart(int n, const double* a, int nkeep, int* r, double* w, double* resid,
                                        int* real_path) {
  if (n < 1 || !a || nkeep < 1 || nkeep > n || !r || !w) return RIGA_ERR_INVALID_ARG;
  std::vector<double> T, Q;
  if (riga::schur_real(n, a, T, Q) != 0) return RIGA_WARN_NOT_CONVERGED;
  // eigenvalue of every diagonal position of the quasi-triangular form
  std::vector<cplx> lam(n);
  for (int i = 0; i < n;) {
    if (i + 1 < n && T[(i + 1) + (size_t)i * n] != 0.0) {
      const double p = T[i + (size_t)i * n], q = T[i + (size_t)(i + 1) * n];
      const double u = T[(i + 1) + (size_t)i * n], v = T[(i + 1) + (size_t)(i + 1) * n];
      const cplx disc = std::sqrt(cplx(0.25 * (p - v) * (p - v) + q * u));
      lam[i] = 0.5 * (p + v) + disc;
      lam[i + 1] = 0.5 * (p + v) - disc;
      i += 2;
    } else {
      lam[i] = T[i + (size_t)i * n];
      i += 1;
    }
  }
  // keep the nkeep of largest modulus, extended to every equal modulus
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return std::abs(lam[x]) > std::abs(lam[y]); });
  int kk = nkeep;
  while (kk < n && std::abs(std::abs(lam[ord[kk]]) - std::abs(lam[ord[kk - 1]])) <= 1e-12 * std::abs(lam[ord[kk - 1]]))
    ++kk;
  std::vector<char> keep(n, 0);
  for (int p = 0; p < kk; ++p) keep[ord[p]] = 1;
  const int rr = riga::schur_select_real(n, T, Q, keep);
  if (real_path) *real_path = rr > 0;
  if (rr <= 0) return RIGA_WARN_NOT_CONVERGED;
  *r = rr;
  // eigenvalues of the leading block and the invariant-subspace residual
  for (int i = 0; i < rr;) {
    if (i + 1 < rr && T[(i + 1) + (size_t)i * n] != 0.0) {
      const double p = T[i + (size_t)i * n], q = T[i + (size_t)(i + 1) * n];
      const double u = T[(i + 1) + (size_t)i * n], v = T[(i + 1) + (size_t)(i + 1) * n];
      const cplx disc = std::sqrt(cplx(0.25 * (p - v) * (p - v) + q * u));
      const cplx l1 = 0.5 * (p + v) + disc, l2 = 0.5 * (p + v) - disc;
      w[2 * i] = l1.real(); w[2 * i + 1] = l1.imag();
      w[2 * i + 2] = l2.real(); w[2 * i + 3] = l2.imag();
      i += 2;
    } else {
      w[2 * i] = T[i + (size_t)i * n]; w[2 * i + 1] = 0.0;
      i += 1;
    }
  }
  double an = 0.0, worst = 0.0;
  for (int i = 0; i < n * n; ++i) an = std::max(an, std::abs(a[i]));
  for (int c = 0; c < rr; ++c)
    for (int i = 0; i < n; ++i) {
      double aq = 0.0, qt = 0.0;
      for (int j = 0; j < n; ++j) aq += a[i + (size_t)j * n] * Q[j + (size_t)c * n];
      for (int j = 0; j < rr; ++j) qt += Q[i + (size_t)j * n] * T[j + (size_t)c * n];
      worst = std::max(worst, std::abs(aq - qt) / std::max(an, 1e-300));
    }
  for (int c = 0; c < rr; ++c)
    for (int d = 0; d < rr; ++d) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += Q[i + (size_t)c * n] * Q[i + (size_t)d * n];
      worst = std::max(worst, std::abs(s - (c == d ? 1.0 : 0.0)));
    }
  if (resid) *resid = worst;
  return RIGA_OK;
}

riga_status riga_time_kernel(riga_problem* h, int which, int nrhs, int reps, double* avg_ms,
                             double* work_per_launch, int* launches) {
  if (!h || which < 0 || which > 2 || nrhs < 1 || nrhs > 4 || reps < 1 || !avg_ms || !work_per_launch)
    return RIGA_ERR_INVALID_ARG;
  if (!h->factored) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    const riga::Plan& P = h->plan;
    const int64_t N = h->N();
    const int H = P.height;
    // a defined right-hand side and forward state for the sweeps
    riga::launch_random_fill(h->d_tmp2, N, nrhs, N, 12345, h->st);
    solve_levels(h, nrhs, h->d_tmp2, N, h->d_tmp2, N, nullptr, nullptr, 0, 0.0);
    double work = 0.0;
    for (int v = 0; v < (int)P.nf.size(); ++v) {
      const double o = P.no[v], b = P.nb[v], f = P.nf[v];
      const double esz = h->level_f32(P.nodes[v].height) ? 4.0 : 8.0;
      if (which == 2) work += o * o * o / 3.0 + b * o * o + b * b * o;
      else work += esz * (o * (o + 1) / 2 + b * o) + 8.0 * nrhs * (f + (which == 0 ? f : o));
    }
    riga::BwdOut o;
    o.xs = h->d_tmp2; o.ldxs = N;
    ck(hipEventRecord(h->ev0, h->st));
    for (int r = 0; r < reps; ++r) {
      for (int lv = 0; lv < H; ++lv) {
        if (which == 0) {
          int a = h->ftask_off[lv], c = h->ftask_off[lv + 1] - a;
          riga::launch_fwd_level(h->dt, h->d_ftasks + a, c, nrhs, h->d_Lp, h->level_f32(lv) ? h->d_Lp32 : nullptr,
                                 h->d_tmp2, N, h->d_tmp, N, h->d_upd, h->lvl_max_nf[lv], h->fvar[lv], h->st);
        } else if (which == 1) {
          int l2 = H - 1 - lv;
          int a = h->btask_off[l2], c = h->btask_off[l2 + 1] - a;
          riga::launch_bwd_level(h->dt, h->d_btasks + a, c, nrhs, h->d_Tp, h->level_f32(l2) ? h->d_Tp32 : nullptr,
                                 h->d_tmp, N, o, h->lvl_max_nf[l2], h->bvar[l2], h->st);
        } else {
          if (h->gep) factor_level(h, lv, -h->sigma, 0.0);
          else factor_level(h, lv, h->sigma * h->sigma, h->sigma);
        }
      }
    }
    ck(hipGetLastError());
    ck(hipEventRecord(h->ev1, h->st));
    ck(hipEventSynchronize(h->ev1));
    float ms = 0;
    ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    *avg_ms = ms / ((double)reps * H);
    *work_per_launch = work / H;
    if (launches) *launches = H;
    return RIGA_OK;
  });
}

riga_status riga_adjoint(riga_problem* h, int nev, const double* lam, const double* X, const double* dL_dlam,
                         double* grad_c) {
  if (!h || nev < 1 || !lam || !X || !dL_dlam || !grad_c) return RIGA_ERR_INVALID_ARG;
  if (!h->assembled) return RIGA_ERR_STATE;
  // the formula needs the complex-symmetric pencil of the scalar space
  if (h->gyro || h->plan.kind != riga::SPACE_H1) return RIGA_ERR_INVALID_ARG;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    const int64_t N = h->N();
    ensure_post(h, nev);
    riga::launch_deinterleave(N, nev, X, h->P, h->st);
    for (int c0 = 0; c0 < 2 * nev; c0 += 8) {
      const int nc = std::min(8, 2 * nev - c0);
      const double* x = h->P + (size_t)c0 * N;
      riga::launch_spmv(h->ds, N, nc, h->d_M, 1.0, x, N, h->MP + (size_t)c0 * N, N,
                        nullptr, 0, 0.0, nullptr, 0, h->st);
      riga::launch_spmv(h->ds, N, nc, h->d_C, 1.0, x, N, h->CP + (size_t)c0 * N, N,
                        nullptr, 0, 0.0, nullptr, 0, h->st);
    }
    const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, N / 4096));
    // the K slots of the pair reduction are not needed: pass M P there
    riga::launch_pair_forms(N, nev, h->P, h->MP, h->CP, h->MP, N, h->d_part, nsplit, h->st);
    std::vector<double> part((size_t)nev * nsplit * 11);
    ck(hipMemcpyAsync(part.data(), h->d_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    std::vector<double> w((size_t)2 * nev);
    for (int k = 0; k < nev; ++k) {
      double f[11] = {0};
      for (int x = 0; x < nsplit; ++x)
        for (int t2 = 0; t2 < 11; ++t2) f[t2] += part[((size_t)k * nsplit + x) * 11 + t2];
      const cplx qm(f[0] - f[1], 2 * f[2]), qc(f[3] - f[4], 2 * f[5]);
      const cplx l(lam[2 * k], lam[2 * k + 1]);
      const cplx den = 2.0 * l * qm + qc;          // u^T (2 lam M + C) u
      const cplx g(dL_dlam[2 * k], dL_dlam[2 * k + 1]);
      const cplx wk = std::conj(g) * (-l / den);
      w[2 * k] = wk.real();
      w[2 * k + 1] = wk.imag();
    }
    double* dw = h->d_part;   // reuse: the reduction scratch is free again
    ck(hipMemcpyAsync(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    riga::launch_adjoint(h->ds, h->d_tabM, nev, h->P, N, dw, grad_c, h->st);
    ck(hipGetLastError());
    ck(hipStreamSynchronize(h->st));
    return RIGA_OK;
  });
}

}  // extern "C"

// =============================================================================
// Block Krylov--Schur on S = L(sigma)^{-1} B (Sec. 4.1.2-4.1.3, Alg. 2).
//
// Basis V = [V_u; V_l] is B-orthonormal, B = diag(I, M); W_l = M V_l is kept
// beside it so that every B-inner product costs no extra sparse product:
//   <x, y>_B = x_u^T y_u + x_l^T M y_l = x_u^T y_u + (M x_l)^T y_l.
// The Krylov decomposition is S V_k = V_{k+b} H, with H (k+b) x k.
// =============================================================================
namespace riga {
namespace detail {

struct KrylovRun {
  riga_problem* h;
  int64_t N;
  int b, m, nev, maxit, ldh;
  double tol;
  std::vector<double> H;   // ldh x ldh, column-major
  int k = 0;               // processed columns
  bool fast = true;        // device-resident normalisation, no host round-trip per step
  bool graphs = true;      // replay captured block steps (fast path only)
  bool pre = false;        // the next step's operator application is already queued
  bool dcgs = false;       // fast path, block <= 2: the second Gram--Schmidt pass delayed by one step
  int64_t n_fb = 0, n_mv = 0, n_vv = 0;

  double& Hat(int r, int c) { return H[r + (size_t)c * ldh]; }

  // B-orthonormalise the block (Ru, Rl, MRl = M Rl) against V[:, 0:nc] by
  // classical Gram--Schmidt applied twice (the coefficients of both passes
  // are summed into hsum, nc x b) and write it to V[:, nc:nc+b] so that
  //   block = V[:, 0:nc] hsum + V[:, nc:nc+b] R.
  // R comes from a Cholesky factorisation of the b x b B-Gram matrix of the
  // projected block.  If the block has lost rank (a column lies in the span of
  // V: an invariant subspace was found), a pivoted factorisation keeps the r
  // independent combinations; the remaining b - r columns of the new block are
  // random directions B-orthogonal to everything, and their rows of R are zero.
  void project(int nc, int nq, double* ru, double* rl, double* mrl, double* dh, std::vector<double>* hsum) {
    const int64_t n = N;
    for (int pass = 0; pass < 2; ++pass) {
      riga::launch_dots(n, nc, h->Vu, h->Wl, n, nq, ru, rl, n, h->d_part, dh + (size_t)pass * ldh * b,
                        h->st);
      riga::launch_cgs_update(n, nc, nq, dh + (size_t)pass * ldh * b, h->Vu, ru, h->Vl, rl, h->Wl, mrl, n, n, nullptr, h->st);
    }
    n_vv += 8LL * nc * nq;
    if (hsum) {
      std::vector<double> host((size_t)2 * ldh * b);
      ck(hipMemcpyAsync(host.data(), dh, host.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
      ck(hipStreamSynchronize(h->st));
      hsum->assign((size_t)nc * nq, 0.0);
      for (int c = 0; c < nc; ++c)
        for (int q = 0; q < nq; ++q)
          (*hsum)[c + (size_t)q * nc] = host[(size_t)c * nq + q] + host[(size_t)ldh * b + (size_t)c * nq + q];
    }
  }

  std::vector<double> gram(int nq, double* ru, double* rl, double* mrl) {
    double* dG = h->d_small + (size_t)2 * ldh * b;
    riga::launch_dots(N, nq, ru, mrl, N, nq, ru, rl, N, h->d_part, dG, h->st);
    n_vv += 2LL * nq * nq;
    std::vector<double> G((size_t)nq * nq);
    ck(hipMemcpyAsync(G.data(), dG, G.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    for (int c = 0; c < nq; ++c)       // symmetrise the two half-sums
      for (int q = c + 1; q < nq; ++q) {
        double v = 0.5 * (G[c + (size_t)q * nq] + G[q + (size_t)c * nq]);
        G[c + (size_t)q * nq] = G[q + (size_t)c * nq] = v;
      }
    return G;
  }

  // Out columns = In (N x kin) times Qm (kin x kout), for the u, l and M l parts.
  void combine(const double* iu, const double* il, const double* iml, int kin, const std::vector<double>& Qm,
               int kout, int dst) {
    double* dQ = h->d_small + (size_t)2 * ldh * b + 32;
    ck(hipMemcpyAsync(dQ, Qm.data(), Qm.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    const size_t o = (size_t)dst * N;
    riga::launch_gemm_tall(N, iu, N, kin, dQ, kout, h->Vu + o, N, h->st);
    riga::launch_gemm_tall(N, il, N, kin, dQ, kout, h->Vl + o, N, h->st);
    riga::launch_gemm_tall(N, iml, N, kin, dQ, kout, h->Wl + o, N, h->st);
    ck(hipStreamSynchronize(h->st));  // dQ is host-staged again by the next call
  }

  // Device path of orthonormalize: same arithmetic, the b x b factor computed by
  // a one-workgroup kernel, H written on the device (dest = nullptr: not recorded).
  // mr: MRl = M Rl is formed here, in the launch of the first products
  void orthonormalize_device(int nc, double* dest, int col, bool mr = false) {
    double* h1 = h->d_small;
    double* h2 = h->d_small + (size_t)ldh * b;
    double* dG = h->d_small + (size_t)2 * ldh * b;
    int gblk = 0;
    if (riga::cgs_tile_fits(nc, b)) {
      // pass 1 products; pass 1 update together with the pass 2 products (one
      // read of the basis); pass 2 update with the partial B-Gram sums of the
      // new block
      if (mr)
        riga::launch_dots_mr(N, nc, h->Vu, h->Wl, N, b, h->Ru, h->Rl, N, h->d_part, h1, h->ds, h->d_M1, h->MRl, N,
                             h->st);
      else
        riga::launch_dots(N, nc, h->Vu, h->Wl, N, b, h->Ru, h->Rl, N, h->d_part, h1, h->st);
      riga::launch_cgs_update_dots(N, nc, b, h1, h->Vu, h->Vl, h->Wl, N, h->Ru, h->Rl, h->MRl, N, h->d_part, h2,
                                   h->st);
      gblk = riga::launch_cgs_update(N, nc, b, h2, h->Vu, h->Ru, h->Vl, h->Rl, h->Wl, h->MRl, N, N, h->d_part,
                                     h->st);
    } else if (nc > 0) {
      if (mr)
        riga::launch_dots_mr(N, nc, h->Vu, h->Wl, N, b, h->Ru, h->Rl, N, h->d_part, h1, h->ds, h->d_M1, h->MRl, N,
                             h->st);
      else
        riga::launch_dots(N, nc, h->Vu, h->Wl, N, b, h->Ru, h->Rl, N, h->d_part, h1, h->st);
      riga::launch_cgs_update(N, nc, b, h1, h->Vu, h->Ru, h->Vl, h->Rl, h->Wl, h->MRl, N, N, nullptr, h->st);
      riga::launch_dots(N, nc, h->Vu, h->Wl, N, b, h->Ru, h->Rl, N, h->d_part, h2, h->st);
      // the second pass also leaves the partial B-Gram sums of the updated block
      gblk = riga::launch_cgs_update(N, nc, b, h2, h->Vu, h->Ru, h->Vl, h->Rl, h->Wl, h->MRl, N, N, h->d_part,
                                     h->st);
    } else {
      riga::launch_dots(N, b, h->Ru, h->MRl, N, b, h->Ru, h->Rl, N, h->d_part, dG, h->st);
    }
    const size_t o = (size_t)nc * N;
    double* rbuf = h->d_small + (size_t)2 * ldh * b + 16;   // nq x nq, after G
    riga::launch_normalize_gemm3(N, nc, b, nc > 0 ? h1 : nullptr, nc > 0 ? h2 : nullptr, dG,
                                 nc > 0 ? h->d_part : nullptr, gblk, dest, ldh, col, h->d_flag, rbuf, h->Ru,
                                 h->Vu + o, h->Rl, h->Vl + o, h->MRl, h->Wl + o, N, h->st);
  }

  void orthonormalize(int nc, std::vector<double>& hsum, std::vector<double>& R, uint64_t seed) {
    double* dh = h->d_small;
    if (nc > 0) project(nc, b, h->Ru, h->Rl, h->MRl, dh, &hsum);
    else hsum.clear();
    std::vector<double> G = gram(b, h->Ru, h->Rl, h->MRl);
    // squared B-norm of each column before the projection (Pythagoras)
    std::vector<double> n0(b);
    for (int q = 0; q < b; ++q) {
      double s = G[q + (size_t)q * b];
      for (int c = 0; c < nc; ++c) s += hsum[c + (size_t)q * nc] * hsum[c + (size_t)q * nc];
      n0[q] = s;
    }
    const double brk = 1e-24;  // (1e-12)^2: relative size of a column that counts as lost
    // Cholesky with symmetric pivoting on the largest remaining diagonal
    std::vector<double> A = G;
    std::vector<int> piv(b);
    std::iota(piv.begin(), piv.end(), 0);
    R.assign((size_t)b * b, 0.0);
    int r = 0;
    std::vector<double> Rp((size_t)b * b, 0.0);  // in pivoted column order
    for (int j = 0; j < b; ++j) {
      int best = j;
      for (int c = j + 1; c < b; ++c)
        if (A[c + (size_t)c * b] / n0[piv[c]] > A[best + (size_t)best * b] / n0[piv[best]]) best = c;
      if (!(A[best + (size_t)best * b] > brk * n0[piv[best]])) break;
      if (best != j) {
        std::swap(piv[j], piv[best]);
        for (int c = 0; c < b; ++c) std::swap(A[j + (size_t)c * b], A[best + (size_t)c * b]);
        for (int c = 0; c < b; ++c) std::swap(A[c + (size_t)j * b], A[c + (size_t)best * b]);
        for (int c = 0; c < j; ++c) std::swap(Rp[c + (size_t)j * b], Rp[c + (size_t)best * b]);
      }
      double d = std::sqrt(A[j + (size_t)j * b]);
      Rp[j + (size_t)j * b] = d;
      for (int c = j + 1; c < b; ++c) Rp[j + (size_t)c * b] = A[j + (size_t)c * b] / d;
      for (int c = j + 1; c < b; ++c)
        for (int q = j + 1; q < b; ++q) A[c + (size_t)q * b] -= Rp[j + (size_t)c * b] * Rp[j + (size_t)q * b];
      ++r;
    }
    // new basis columns nc .. nc+r-1 = block[:, piv[0:r]] R11^{-1}
    if (r > 0) {
      std::vector<double> R11((size_t)r * r);
      for (int c = 0; c < r; ++c)
        for (int q = 0; q < r; ++q) R11[c + (size_t)q * r] = Rp[c + (size_t)q * b];
      std::vector<double> Ri = upper_inverse(r, R11);
      std::vector<double> Qm((size_t)b * r, 0.0);
      for (int c = 0; c < r; ++c)
        for (int j = 0; j < r; ++j) Qm[piv[c] + (size_t)j * b] = Ri[c + (size_t)j * r];
      combine(h->Ru, h->Rl, h->MRl, b, Qm, r, nc);
    }
    // R[c][q] = Rp[c][position of q]: block column q = sum_c newV_c R[c][q]
    for (int pos = 0; pos < b; ++pos)
      for (int c = 0; c < r; ++c) R[c + (size_t)piv[pos] * b] = Rp[c + (size_t)pos * b];
    if (r < b) {
      // fresh random directions, B-orthogonal to V[:, 0:nc+r]
      const int nf = b - r;
      riga::launch_random_fill(h->Ru, N, nf, N, seed * 7919u + 17u, h->st);
      riga::launch_random_fill(h->Rl, N, nf, N, seed * 7919u + 29u, h->st);
      riga::launch_spmv(h->ds, N, nf, h->d_M, 1.0, h->Rl, N, h->MRl, N, nullptr, 0, 0.0,
                        nullptr, 0, h->st);
      project(nc + r, nf, h->Ru, h->Rl, h->MRl, dh, nullptr);
      std::vector<double> Gf = gram(nf, h->Ru, h->Rl, h->MRl);
      std::vector<double> Rf;
      small_chol(nf, Gf, Rf, 0.0);
      combine(h->Ru, h->Rl, h->MRl, nf, upper_inverse(nf, Rf), nf, nc + r);
    }
  }

  // One block step on the device: S applied to V[:, k:k+b], CGS2 against
  // V[:, 0:k+b], device normalisation into V[:, k+b:k+2b] and H.
  // The operator applied to the basis block at column kb: Ru, Rl (M Rl is
  // formed by orthonormalize_device, with the first products).
  void enqueue_apply(int kb) {
    const int64_t n = N;
    const size_t o = (size_t)kb * n;
    apply_block(h, b, h->Vu + o, h->Wl + o, n, h->Ru, h->Rl, h->Tv);
  }

  // Scratch of the delayed-pass steps in d_small: the products P ((k+b) x 2b)
  // where the two pass coefficients lie otherwise, then the update
  // coefficients and T^{-1}.
  double* dcgs_P() { return h->d_small; }
  double* dcgs_hc() { return h->d_small + (size_t)2 * ldh * b + 64; }
  double* dcgs_Xm() { return dcgs_hc() + (size_t)2 * ldh * b; }

  // One block step with the delayed second pass: the pending block Y =
  // V[:, k:k+b] is finished (second pass and normalisation) and W = S Y
  // projected once against [V[:, 0:k] V_j] in two reads of the basis; the
  // projected image is the next pending block V[:, k+b:k+2b] as it stands.
  void dcgs_step_device(bool tensor) {
    riga::launch_dcgs_dots(N, k, b, true, h->Vu, h->Vl, h->Wl, N, h->Ru, h->Rl, h->d_part, dcgs_P(),
                           tensor ? &h->ds : nullptr, h->d_M1, h->MRl, h->st);
    riga::launch_dcgs_coef(k, b, true, dcgs_P(), h->d_H, ldh, dcgs_hc(), dcgs_Xm(), h->d_flag, h->st);
    riga::launch_dcgs_update(N, k, b, true, dcgs_hc(), dcgs_Xm(), h->Vu, h->Vl, h->Wl, N, h->Ru, h->Rl, h->MRl, N,
                             h->st);
  }

  // The second pass of the last block V[:, k:k+b] (end of a cycle, before the
  // projected matrix is read), with H's columns rewritten for it.
  void dcgs_finish_device() {
    riga::launch_dcgs_dots(N, k, b, false, h->Vu, h->Vl, h->Wl, N, nullptr, nullptr, h->d_part, dcgs_P(), nullptr,
                           nullptr, nullptr, h->st);
    riga::launch_dcgs_coef(k, b, false, dcgs_P(), h->d_H, ldh, dcgs_hc(), nullptr, h->d_flag, h->st);
    riga::launch_dcgs_update(N, k, b, false, dcgs_hc(), nullptr, h->Vu, h->Vl, h->Wl, N, nullptr, nullptr, nullptr,
                             N, h->st);
    n_vv += 5LL * (k + b) * b;
  }

  // (M Rl, which the Gram-Schmidt updates need, is formed with the first products)
  void enqueue_step_device() {
    if (!pre) enqueue_apply(k);
    const bool tensor = h->plan.kind == riga::SPACE_H1;
    if (!tensor)
      riga::launch_spmv(h->ds, N, b, h->d_M, 1.0, h->Rl, N, h->MRl, N, nullptr, 0, 0.0, nullptr, 0, h->st);
    if (dcgs) dcgs_step_device(tensor);
    else orthonormalize_device(k + b, h->d_H, k, tensor);
  }

  void step(uint64_t seed) {
    const int64_t n = N;
    const size_t o = (size_t)k * n;
    const int nc = k + b;
    if (fast) {
      if (graphs) {
        auto key = std::make_tuple(k, b, (const double*)h->Vu, (pre ? 1 : 0) + (dcgs ? 2 : 0), ldh);
        auto it = h->graphs.find(key);
        if (it == h->graphs.end()) {
          ck(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
          enqueue_step_device();
          hipGraph_t g = nullptr;
          ck(hipStreamEndCapture(h->st, &g));
          hipGraphExec_t ex = nullptr;
          hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
          hipGraphDestroy(g);
          ck(e);
          it = h->graphs.emplace(key, ex).first;
        }
        ck(hipGraphLaunch(it->second, h->st));
      } else {
        enqueue_step_device();
      }
      pre = false;
      n_fb += b;
      n_mv += 3LL * b;
      n_vv += (dcgs ? 10LL : 8LL) * nc * b + 2LL * b * b;
      k += b;
      return;
    }
    apply_block(h, b, h->Vu + o, h->Wl + o, n, h->Ru, h->Rl, h->Tv);
    riga::launch_spmv(h->ds, n, b, h->d_M, 1.0, h->Rl, n, h->MRl, n, nullptr, 0, 0.0,
                      nullptr, 0, h->st);
    n_fb += b;
    n_mv += 3LL * b;
    {
      std::vector<double> hs, R;
      orthonormalize(nc, hs, R, seed);
      for (int q = 0; q < b; ++q) {
        for (int c = 0; c < nc; ++c) Hat(c, k + q) = hs[c + (size_t)q * nc];
        for (int c = 0; c < b; ++c) Hat(nc + c, k + q) = R[c + (size_t)q * b];
      }
    }
    k += b;
  }
};

// Eigenpairs from the planar Ritz vectors of the wanted values in h->P
// (N x 2 nw: real parts, then imaginary parts; nw = cyc.wanted.size()):
// Rayleigh polish of each value (the root of u^T Q(lam) u = 0 nearest the
// Ritz value), explicit scaled residuals, canonical order, and the normalised
// eigenvectors written to X.  dsmall: device scratch of >= 3 nev + 2 nw + 16
// doubles.  Returns the number of leading pairs (canonical order) whose
// residual meets kEtaConverged.
int finish_pairs(riga_problem* h, const riga::KsCycle& cyc, int nev, double* dsmall, double* lam, double* X,
                 double* eta) {
  const int64_t N = h->N();
  const std::vector<int>& wanted = cyc.wanted;
  const int nw = (int)wanted.size();
    // M, C, K times the planar real and imaginary parts
    for (int c0 = 0; c0 < 2 * nw; c0 += 8) {
      int nc = std::min(8, 2 * nw - c0);
      const double* x = h->P + (size_t)c0 * N;
      riga::launch_spmv3(h->ds, N, nc, h->d_M, h->d_C, h->d_K, x, N, h->MP + (size_t)c0 * N, h->CP + (size_t)c0 * N,
                         h->KP + (size_t)c0 * N, N, h->st);
    }
    const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, N / 4096));
    riga::launch_pair_forms(N, nw, h->P, h->MP, h->CP, h->KP, N, h->d_part, nsplit, h->st);
    std::vector<double> part((size_t)nw * nsplit * 11);
    ck(hipMemcpyAsync(part.data(), h->d_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    // with a skew part in C the pencil is not complex-symmetric: the polish
    // takes the root of u^H Q(lam) u = 0 instead, which needs b^T C a besides
    std::vector<double> cross;
    if (h->gyro) {
      riga::launch_cross_form(N, nw, h->P, h->CP, N, h->d_part + (size_t)nw * nsplit * 11, nsplit, h->st);
      cross.resize((size_t)nw * nsplit);
      ck(hipMemcpyAsync(cross.data(), h->d_part + (size_t)nw * nsplit * 11, cross.size() * sizeof(double),
                        hipMemcpyDeviceToHost, h->st));
      ck(hipStreamSynchronize(h->st));
    }
    std::vector<cplx> lam_rq(nw);
    std::vector<double> uMu(nw), unorm2(nw);
    for (int j = 0; j < nw; ++j) {
      double f[11] = {0};
      for (int x = 0; x < nsplit; ++x)
        for (int t2 = 0; t2 < 11; ++t2) f[t2] += part[((size_t)j * nsplit + x) * 11 + t2];
      riga::PairForms pf = riga::pair_forms(f);
      uMu[j] = pf.uMu;
      unorm2[j] = pf.unorm2;
      if (h->gyro) {
        double g = 0.0;
        for (int x = 0; x < nsplit; ++x) g += cross[(size_t)j * nsplit + x];
        pf.qm = cplx(f[0] + f[1], 0.0);          // u^H M u
        pf.qc = cplx(f[3] + f[4], f[5] - g);     // u^H C u
        pf.qk = cplx(f[6] + f[7], 0.0);          // u^H K u
      }
      lam_rq[j] = h->cmode ? cshift_polish(pf, cyc.theta[wanted[j]], h->sigma, h->csig_im)
                           : riga::rayleigh_polish(pf, h->sigma + 1.0 / cyc.theta[wanted[j]]);
    }
    std::vector<double> lamd((size_t)2 * nw);
    for (int j = 0; j < nw; ++j) { lamd[2 * j] = lam_rq[j].real(); lamd[2 * j + 1] = lam_rq[j].imag(); }
    double* dlam = dsmall + 8;
    ck(hipMemcpyAsync(dlam, lamd.data(), lamd.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    riga::launch_pair_resid(N, nw, h->P, h->MP, h->CP, h->KP, N, dlam, h->d_part, nsplit, h->st);
    std::vector<double> rpart((size_t)nw * nsplit * 5);
    ck(hipMemcpyAsync(rpart.data(), h->d_part, rpart.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    std::vector<double> etav(nw);
    std::vector<cplx> umax(nw);
    for (int j = 0; j < nw; ++j) {
      double s = 0.0, best = -1.0;
      for (int x = 0; x < nsplit; ++x) {
        const double* o = &rpart[((size_t)j * nsplit + x) * 5];
        s += o[0];
        if (o[1] > best) { best = o[1]; umax[j] = cplx(o[3], o[4]); }
      }
      etav[j] = riga::scaled_residual(s, lam_rq[j], h->norms, unorm2[j]);
    }
    std::vector<int> order = h->cmode ? psi_order(lam_rq, h->sigma, h->csig_im) : canonical_order(lam_rq, h->sigma);
    const int nout = std::min(nev, nw);
    // converged pairs: the leading ones in canonical order whose explicit
    // scaled residual meets the bar (the Ritz estimate alone is not trusted)
    int conv_out = 0;
    for (int j = 0; j < nout; ++j) {
      if (etav[order[j]] <= riga::detail::kEtaConverged) ++conv_out; else break;
    }
    for (int j = 0; j < nout; ++j) {
      lam[2 * j] = lam_rq[order[j]].real();
      lam[2 * j + 1] = lam_rq[order[j]].imag();
      if (eta) eta[j] = etav[order[j]];
    }
    if (X) {
      // scale u^H M u = 1 with an entry of largest modulus real positive, in output order
      std::vector<double> sc((size_t)3 * nout);
      for (int j = 0; j < nout; ++j) {
        const int src = order[j];
        const cplx ph = std::conj(umax[src]) / std::abs(umax[src]);
        const cplx s = ph / std::sqrt(uMu[src]);
        sc[3 * j] = s.real();
        sc[3 * j + 1] = s.imag();
        sc[3 * j + 2] = (double)src;
      }
      double* dsc = dsmall + 8;
      double* stage = h->pinned(sc.size() + 8);
      std::memcpy(stage, sc.data(), sc.size() * sizeof(double));
      ck(hipMemcpyAsync(dsc, stage, sc.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
      riga::launch_finalize(N, nw, nout, h->P, N, dsc, X, h->st);
    }
  return conv_out;
}

}  // namespace detail
}  // namespace riga

extern "C" riga_status riga_eigs(riga_problem* h, const riga_options* opt, double* lam, double* X,
                                 double* eta, int* nconv) {
  if (!h || !opt || !lam) return RIGA_ERR_INVALID_ARG;
  // a real shift on a vector space would return its gradients (lam = 0 and
  // -alpha are nearest every positive shift); a complex target is taken
  if (h->plan.kind != riga::SPACE_H1 && !h->cmode) return RIGA_ERR_INVALID_ARG;
  if ((!h->factored || h->gep) && !h->cmode) return RIGA_ERR_STATE;
  if (h->cmode && (opt->flags & RIGA_EIGS_TOAR)) return RIGA_ERR_INVALID_ARG;
  const int64_t N = h->N();
  const int nev = opt->nev;
  const int b = opt->block > 0 ? opt->block : 2;
  int m = opt->m > 0 ? opt->m : std::max(2 * nev, 20);
  const int maxit = opt->maxit > 0 ? opt->maxit : 200;
  const double tol = opt->tol > 0 ? opt->tol : 1e-12;
  if (nev < 1 || b < 1 || b > 4 || (int64_t)nev >= 2 * N) return RIGA_ERR_INVALID_ARG;
  if ((int64_t)m > 2 * N) m = (int)(2 * N);
  if (m < nev + b || m + 2 * b > 256 || opt->keep < 0 || opt->keep > m - b) return RIGA_ERR_INVALID_ARG;
  // the solve runs on the handle's own stream, fenced to the caller's stream
  hipStream_t user_st = h->st;
  struct Restore {
    riga_problem* h; hipStream_t s;
    ~Restore() { h->st = s; }
  } restore{h, user_st};
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    ck(hipEventRecord(h->ev_fence, user_st));
    ck(hipStreamWaitEvent(h->own_st, h->ev_fence, 0));
    h->st = h->own_st;
    if (h->graph_sigma != h->sigma || h->graph_key != h->factor_key()) {
      h->clear_graphs();
      h->graph_sigma = h->sigma;
      h->graph_key = h->factor_key();
    }
    ensure_norms(h);
    h->stats.toar_drop = 0.0;
    if (opt->flags & RIGA_EIGS_TOAR) {
      bool fallback = false;
      const riga_status rs = eigs_toar(h, opt, nev, b, m, maxit, tol, lam, X, eta, nconv, &fallback);
      if (!fallback) return rs;
      h->stats.toar_drop = 0.0;
    }
    const int ldh = m + 2 * b;
    ensure_krylov(h, ldh, b);
    ck(hipEventRecord(h->ev0, h->st));
    KrylovRun kr{h, N, b, m, nev, maxit, ldh, tol};
    int it = 0;
    bool converged = false;
    double t_host = 0.0;   // host Ritz and restart work, the device idle
    double rs_bytes = 0.0, rs_flops = 0.0;   // restart recombinations
    riga::KsCycle cyc;
    uint64_t step_seed = opt->seed * 1000003u + 5;
    // First attempt on the fast path; a breakdown reported by the device sends
    // the solve once more through the host-checked path.
    for (int attempt = 0; attempt < 2; ++attempt) {
    kr.fast = (attempt == 0) && !(opt->flags & 2);
    kr.graphs = !(opt->flags & 1);
    kr.dcgs = kr.fast && b <= 2 && !(opt->flags & RIGA_EIGS_CGS2);
    if (!kr.fast && attempt == 0) attempt = 1;
    kr.H.assign((size_t)ldh * ldh, 0.0);
    kr.n_fb = kr.n_mv = kr.n_vv = 0;
    kr.pre = false;
    it = 0;
    converged = false;
    step_seed = opt->seed * 1000003u + 5;
    ck(hipMemsetAsync(h->d_flag, 0, sizeof(int), h->st));
    ck(hipMemsetAsync(h->d_H, 0, sizeof(double) * (size_t)ldh * ldh, h->st));
    // start block, B-orthonormalised
    if (opt->v0) {
      for (int q = 0; q < b; ++q) {
        ck(hipMemcpyAsync(h->Ru + (size_t)q * N, opt->v0 + (size_t)q * 2 * N, N * sizeof(double),
                          hipMemcpyDeviceToDevice, h->st));
        ck(hipMemcpyAsync(h->Rl + (size_t)q * N, opt->v0 + (size_t)q * 2 * N + N, N * sizeof(double),
                          hipMemcpyDeviceToDevice, h->st));
      }
    } else {
      riga::launch_random_fill(h->Ru, N, b, N, opt->seed * 2 + 1, h->st);
      riga::launch_random_fill(h->Rl, N, b, N, opt->seed * 2 + 2, h->st);
    }
    riga::launch_spmv(h->ds, N, b, h->d_M, 1.0, h->Rl, N, h->MRl, N, nullptr, 0, 0.0,
                      nullptr, 0, h->st);
    if (kr.fast) {
      kr.orthonormalize_device(0, nullptr, 0);
    } else {
      std::vector<double> hs, R;
      kr.orthonormalize(0, hs, R, opt->seed + 99);
    }
    kr.k = 0;
    bool broke = false;
    for (;;) {
      while (kr.k + b <= m) kr.step(step_seed++);
      if (kr.dcgs) kr.dcgs_finish_device();
      if (kr.fast) {
        const size_t hl = (size_t)ldh * ldh;
        double* stage = h->pinned(3 * hl + 8);   // the size the restart stages with
        ck(hipMemcpyAsync(stage, h->d_H, sizeof(double) * hl, hipMemcpyDeviceToHost, h->st));
        ck(hipMemcpyAsync(stage + 2 * hl, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->st));
        ck(hipStreamSynchronize(h->st));
        std::memcpy(kr.H.data(), stage, sizeof(double) * hl);
        int flag = 0;
        std::memcpy(&flag, stage + 2 * hl, sizeof(int));
        if (flag) { broke = true; break; }
      }
      const int k = kr.k;
      // The first step after a restart applies the operator to the last block,
      // which the restart keeps unchanged (column r of the new basis is column k
      // of this one): queue that application now, on the current buffers, so
      // the device computes it while the host forms the Ritz values.  It is
      // discarded when the iteration stops here.
      if (kr.fast) {
        kr.enqueue_apply(k);
        kr.pre = true;
      }
      const auto th0 = std::chrono::steady_clock::now();   // the device waits from here
      if (riga::ks_ritz(kr.H, ldh, k, b, nev, tol, cyc) != 0) throw HipError{hipErrorUnknown};
      ++it;
      if (cyc.nconv == cyc.nw || it >= maxit) {
        t_host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
        converged = cyc.nconv == cyc.nw;
        break;
      }
      // --- Krylov--Schur restart: keep the nearest Ritz values ------------------
      riga::ks_restart(kr.H, ldh, k, b, m, nev, opt->keep, cyc);
      const int r = cyc.r;
      // V_new = [V_k Qk, V_{k:k+b}] in the alternate buffers
      const int kin = k + b, kout = r + b;
      double* dQ = h->d_small;
      // pinned staging: the combination in the first 2 ldh^2 doubles, the new
      // projected matrix after it (both copies complete, in stream order,
      // before the next cycle's download reuses the block)
      const size_t hl2 = (size_t)ldh * ldh;
      double* stage = h->pinned(3 * hl2 + 8);
      std::memcpy(stage, cyc.Qe.data(), cyc.Qe.size() * sizeof(double));
      ck(hipMemcpyAsync(dQ, stage, cyc.Qe.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
      riga::launch_gemm_tall(N, h->Vu, N, kin, dQ, kout, h->Vu2, N, h->st);
      riga::launch_gemm_tall(N, h->Vl, N, kin, dQ, kout, h->Vl2, N, h->st);
      riga::launch_gemm_tall(N, h->Wl, N, kin, dQ, kout, h->Wl2, N, h->st);
      rs_bytes += 3.0 * 8.0 * (double)N * (kin + kout);
      rs_flops += 3.0 * 2.0 * (double)N * kin * kout;
      std::swap(h->Vu, h->Vu2); std::swap(h->Vl, h->Vl2); std::swap(h->Wl, h->Wl2);
      kr.H = cyc.Hn;
      t_host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
      if (kr.fast) {
        std::memcpy(stage + 2 * hl2, kr.H.data(), sizeof(double) * hl2);
        ck(hipMemcpyAsync(h->d_H, stage + 2 * hl2, sizeof(double) * hl2, hipMemcpyHostToDevice, h->st));
      } else {
        ck(hipStreamSynchronize(h->st));   // the host path stages its own copies next
      }
      kr.k = r;
    }
    if (!broke) break;
    }  // attempts
    // --- eigenpairs: u = V_u y for the wanted Ritz vectors --------------------------
    const int k = kr.k;
    riga::ks_ritz_vectors(cyc);
    const std::vector<int>& wanted = cyc.wanted;
    const int nw = (int)wanted.size();
    std::vector<double> Yr((size_t)k * nw), Yi((size_t)k * nw);
    for (int j = 0; j < nw; ++j)
      for (int c = 0; c < k; ++c) {
        cplx y = cyc.Y[c + (size_t)wanted[j] * k];
        Yr[c + (size_t)j * k] = y.real();
        Yi[c + (size_t)j * k] = y.imag();
      }
    ensure_post(h, nw);
    double* dQ = h->d_small;
    ck(hipMemcpyAsync(dQ, Yr.data(), Yr.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    riga::launch_gemm_tall(N, h->Vu, N, k, dQ, nw, h->P, N, h->st);
    ck(hipStreamSynchronize(h->st));
    ck(hipMemcpyAsync(dQ, Yi.data(), Yi.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    riga::launch_gemm_tall(N, h->Vu, N, k, dQ, nw, h->P + (size_t)nw * N, N, h->st);
    const int conv_out = finish_pairs(h, cyc, nev, h->d_small, lam, X, eta);
    ck(hipEventRecord(h->ev1, h->st));
    ck(hipStreamSynchronize(h->st));
    float ms = 0;
    ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->stats.t_eigs_ms = ms;
    h->stats.n_it = it;
    h->stats.n_fb = kr.n_fb;
    h->stats.t_host_ms = t_host;
    h->stats.n_ir = h->mixed ? kr.n_fb * h->ir_sweeps : 0;
    h->stats.n_mv = kr.n_mv + h->stats.n_ir;   // one residual product per refinement sweep
    h->stats.n_vv = kr.n_vv;
    {
      // algorithmic work per phase (eq. Cost; the byte model is stated with riga_stats_t)
      riga_stats_t& S = h->stats;
      riga::Plan& Pm = h->plan;
      Pm.ensure_symbolic();
      const double Nd = (double)N, nnz = (double)Pm.nnz, irs = h->mixed ? h->ir_sweeps : 0;
      const double vec = (double)kr.n_fb;                 // vectors through the operator
      const double passes = vec / b * (1.0 + irs);        // sweep passes over the factor
      S.bytes[RIGA_PHASE_FB] = passes * h->solve_bytes_now + vec * (1.0 + irs) * 16.0 * Nd;
      // (a complex target: the real form's two dense triangles, 2 flops per entry and vector)
      S.flops[RIGA_PHASE_FB] = h->cmode ? vec * 2.0 * h->solve_bytes_now / 8.0
                                        : vec * (1.0 + irs) * 4.0 * (double)Pm.sym_nnz_l;
      const double mv_bytes = 16.0 * Nd + (h->c_elem ? 8.0 * nnz + 16.0 * Nd : 16.0 * Nd);
      S.bytes[RIGA_PHASE_MV] = vec * mv_bytes;
      S.flops[RIGA_PHASE_MV] = (double)kr.n_mv * 2.0 * nnz;
      S.bytes[RIGA_PHASE_VV] = (double)kr.n_vv * 8.0 * Nd;
      S.flops[RIGA_PHASE_VV] = (double)kr.n_vv * 2.0 * Nd;
      S.bytes[RIGA_PHASE_RESTART] = rs_bytes + 2.0 * 8.0 * Nd * (k + nw);
      S.flops[RIGA_PHASE_RESTART] = rs_flops + 2.0 * 2.0 * Nd * k * nw;
      S.bytes[RIGA_PHASE_IR] = passes > 0 && irs > 0 ? vec / b * irs * 8.0 * nnz + vec * irs * 24.0 * Nd : 0.0;
      S.flops[RIGA_PHASE_IR] = vec * irs * 2.0 * nnz;
      const double pv = 2.0 * nw;                         // planar real / imaginary parts
      S.bytes[RIGA_PHASE_POST] = std::ceil(pv / 8.0) * 24.0 * nnz + pv * 32.0 * Nd;
      S.flops[RIGA_PHASE_POST] = pv * 3.0 * 2.0 * nnz;
    }
    if (nconv) *nconv = conv_out;
    return (converged && conv_out == nev) ? RIGA_OK : RIGA_WARN_NOT_CONVERGED;
  });
}
