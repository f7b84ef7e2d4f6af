// Batched form: many independent damped-wave QEPs of different sizes (degree,
// mesh, damping, shift) factored and solved together on one device.
//
// The problems' nested-dissection trees are merged into one forest (tree
// levels grouped by height across problems), so every factorization level and
// every forward/backward sweep is one set of launches for all of them.  The
// Krylov--Schur iterations (Alg. 2 per problem) run in lockstep: per-problem
// state (current column, live flag, projected matrix) is kept on the device and
// one block step of every problem is a single captured HIP graph replayed for
// the whole cycle; the host only sees the projected matrices at cycle ends,
// where each problem gets its own Ritz values, convergence test and restart.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>

#include "ks_host.hpp"
#include "host_pool.hpp"
#include "problem.hpp"

using riga::cplx;
using namespace riga::detail;

struct riga_batch {
  int n = 0;
  int device = 0;
  hipStream_t user_st = nullptr;
  std::vector<riga_mesh> meshes;
  std::vector<riga::Plan> plans;
  riga_problem* fp = nullptr;            // the forest: CSR values, factor, sweep tasks
  std::vector<int64_t> dof_base;         // n + 1
  const int64_t* d_nzbase = nullptr;     // per problem: first nonzero of its rows (n + 1)
  std::vector<int> node_base;            // n + 1
  std::vector<riga::DevSpace> hsp;       // per problem (device pointers)
  std::vector<double*> tabM, tabK, gx, gw;
  std::vector<double> alpha, beta, sigma;
  std::vector<const double*> celem;
  std::vector<double> norms;             // per problem ||K||_1, ||C||_1, ||M||_1
  std::vector<int> rb_problem;           // problem of every row block
  // batched assembly: tables, Gauss rules and damping per problem (device)
  int max_ne = 0;
  const int64_t* d_taboff = nullptr;
  const double* const* d_gx = nullptr;
  const double* const* d_gw = nullptr;
  double *d_tabM = nullptr, *d_tabK = nullptr, *d_alpha = nullptr, *d_beta = nullptr;
  const double** d_celem = nullptr;
  // sum-factorised products: grid tiles of every problem, banded 1-D factors
  const int4* d_ttiles = nullptr;
  int nttiles = 0, max_p = 0, max_w = 0;
  const int64_t* d_bandoff = nullptr;
  double *d_M1 = nullptr, *d_K1 = nullptr;
  bool any_field = false;                 // some problem has an element damping field
  bool assembled = false, factored = false;
  riga::BatchDev B{};
  // Krylov workspace
  int kw_ldh = 0, kw_b = 0;
  double *Vu = nullptr, *Vl = nullptr, *Wl = nullptr, *Vu2 = nullptr, *Vl2 = nullptr, *Wl2 = nullptr;
  double *Ru = nullptr, *Rl = nullptr, *MRl = nullptr, *Tv = nullptr, *Xu = nullptr, *Xw = nullptr;
  double *h1 = nullptr, *h2 = nullptr, *G = nullptr, *Rinv = nullptr, *H = nullptr, *Qd = nullptr;
  double *P = nullptr, *MP = nullptr, *CP = nullptr, *KP = nullptr, *part = nullptr, *dlam = nullptr;
  int *kin = nullptr, *kout = nullptr;
  int *kin_f = nullptr, *kout_f = nullptr;   // Ritz-vector products of the problems that finish
  int64_t* qoff = nullptr;
  std::map<const double*, hipGraphExec_t> graphs;  // one block step per basis buffer
  int graph_b = 0, graph_m = 0;                    // step shape the graphs were captured for
  int n_broke = 0;                                 // problems re-solved one by one in the last call
  riga_stats_t stats{};

  int64_t N(int p) const { return dof_base[p + 1] - dof_base[p]; }
  void clear_graphs() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
};

namespace {

template <class F>
void parallel_for(int n, F f) {
  riga::HostPool::get().run(n, std::function<void(int)>(f));
}

constexpr int DOT_ROWS = 2048;   // rows per dot block

void ensure_workspace(riga_batch* bh, int ldh, int b) {
  if (bh->kw_ldh >= ldh && bh->kw_b >= b) return;
  riga_problem* fp = bh->fp;
  bh->clear_graphs();
  for (double* p : {bh->Vu, bh->Vl, bh->Wl, bh->Vu2, bh->Vl2, bh->Wl2, bh->Ru, bh->Rl, bh->MRl, bh->Tv,
                    bh->Xu, bh->Xw, bh->h1, bh->h2, bh->G, bh->Rinv, bh->H, bh->Qd, bh->P, bh->MP, bh->CP, bh->KP,
                    bh->part, bh->dlam, bh->B.partial})
    fp->dfree(p);
  fp->dfree(bh->kin); fp->dfree(bh->kout); fp->dfree(bh->qoff);
  fp->dfree(bh->kin_f); fp->dfree(bh->kout_f);
  ldh = std::max(ldh, bh->kw_ldh);
  b = std::max(b, bh->kw_b);
  const int64_t T = bh->B.ntot;
  const int n = bh->n;
  bh->Vu = fp->dalloc<double>(T * ldh); bh->Vl = fp->dalloc<double>(T * ldh); bh->Wl = fp->dalloc<double>(T * ldh);
  bh->Vu2 = fp->dalloc<double>(T * ldh); bh->Vl2 = fp->dalloc<double>(T * ldh);
  bh->Wl2 = fp->dalloc<double>(T * ldh);
  for (double** p : {&bh->Ru, &bh->Rl, &bh->MRl, &bh->Tv, &bh->Xu, &bh->Xw}) *p = fp->dalloc<double>(T * b);
  bh->h1 = fp->dalloc<double>((size_t)n * ldh * b);
  bh->h2 = fp->dalloc<double>((size_t)n * ldh * b);
  bh->G = fp->dalloc<double>((size_t)n * b * b);
  bh->Rinv = fp->dalloc<double>((size_t)n * b * b);
  bh->H = fp->dalloc<double>((size_t)n * ldh * ldh);
  bh->Qd = fp->dalloc<double>((size_t)n * 2 * ldh * ldh);   // Ritz vectors: k x 2 nw per problem
  for (double** p : {&bh->P, &bh->MP, &bh->CP, &bh->KP}) *p = fp->dalloc<double>(T * 2 * ldh);
  bh->part = fp->dalloc<double>((size_t)n * 2 * ldh * 64 * 11 + 64);
  bh->dlam = fp->dalloc<double>((size_t)n * 2 * ldh);
  bh->kin = fp->dalloc<int>(n);
  bh->kout = fp->dalloc<int>(n);
  bh->kin_f = fp->dalloc<int>(n);
  bh->kout_f = fp->dalloc<int>(n);
  bh->qoff = fp->dalloc<int64_t>(n);
  bh->B.pstride = ldh * 4;
  bh->B.partial = fp->dalloc<double>((size_t)bh->B.ndb * bh->B.pstride);
  bh->kw_ldh = ldh;
  bh->kw_b = b;
}

// One block step of every live problem (see the file comment).
void enqueue_step(riga_batch* bh, int b, int m, int ldh, hipStream_t st) {
  riga_problem* fp = bh->fp;
  const riga::BatchDev& B = bh->B;
  const int64_t T = B.ntot;
  const int hs = ldh * b;
  riga::launch_gather_b(B, b, bh->Vu, bh->Wl, bh->Xu, bh->Xw, st);
  // t = (sigma M + C) v_u + M v_l (eq. BlockOperatorVector): sum-factorised with
  // sigma M + C = (sigma + alpha) M + beta K, or the per-problem sparse copy of
  // sigma M + C when a problem carries an element damping field
  if (bh->any_field)
    riga::launch_spmv_ell(fp->d_slabs, fp->nslab, B.spaces, B.dofbase, B.live, b, fp->d_Aell, bh->Xu, T, bh->Tv, T,
                          bh->Xw, T, 1.0, st);
  else
    riga::launch_tensor_mk_b(bh->d_ttiles, bh->nttiles, B.spaces, B.dofbase, bh->d_bandoff, bh->d_M1, bh->d_K1,
                             B.live, B.sig, bh->d_alpha, bh->d_beta, b, bh->max_p, bh->Xu, T, bh->Tv, T, bh->Xw, T,
                             1.0, st);
  // r_u = -Q^{-1} t, r_l = sigma r_u + v_u (sigma of each node's problem)
  riga::BwdOut o;
  o.xs = bh->Ru; o.ldxs = T; o.neg = 1; o.ldr = T;
  o.rl = bh->Rl; o.v_u = bh->Xu; o.ldv = T;
  sweep(fp, b, bh->Tv, T, o);
  riga::launch_tensor_mk_b(bh->d_ttiles, bh->nttiles, B.spaces, B.dofbase, bh->d_bandoff, bh->d_M1, bh->d_K1, B.live,
                           nullptr, nullptr, nullptr, b, bh->max_p, bh->Rl, T, bh->MRl, T, nullptr, 0, 0.0, st);
  // classical Gram--Schmidt twice against V[:, 0:k+b], B-inner products; where
  // the tile kernels fit, the pass 1 update also forms the pass 2 products
  if (riga::cgs_tile_fits(m + b, b)) {
    riga::launch_cgs_dots_tile_b(B, b, b, m + b, bh->Vu, bh->Wl, bh->Ru, bh->Rl, bh->h1, hs, st);
    riga::launch_cgs_update_dots_b(B, b, b, m + b, bh->h1, hs, bh->Vu, bh->Vl, bh->Wl, bh->Ru, bh->Rl, bh->MRl,
                                   bh->h2, hs, st);
  } else {
    riga::launch_dots_b(B, b, 0, true, bh->Vu, bh->Wl, b, bh->Ru, bh->Rl, bh->h1, hs, st);
    riga::launch_cgs_update_b(B, b, b, bh->h1, hs, bh->Vu, bh->Ru, bh->Vl, bh->Rl, bh->Wl, bh->MRl, m + b, st);
    riga::launch_dots_b(B, b, 0, true, bh->Vu, bh->Wl, b, bh->Ru, bh->Rl, bh->h2, hs, st);
  }
  riga::launch_cgs_update_b(B, b, b, bh->h2, hs, bh->Vu, bh->Ru, bh->Vl, bh->Rl, bh->Wl, bh->MRl, m + b, st);
  riga::launch_dots_b(B, 0, b, false, bh->Ru, bh->MRl, b, bh->Ru, bh->Rl, bh->G, b * b, st);
  riga::launch_block_normalize_b(B, true, b, b, bh->h1, bh->h2, hs, bh->G, bh->H, ldh, bh->Rinv, st);
  riga::launch_gemm3_b(B, true, b, b, bh->Rinv, bh->Ru, bh->Vu, bh->Rl, bh->Vl, bh->MRl, bh->Wl, st);
  riga::launch_advance_b(B, b, m, st);
}

}  // namespace

extern "C" {

riga_status riga_batch_create(riga_batch** out, int n, const riga_mesh* meshes, int device, void* hip_stream) {
  if (!out || n < 1 || !meshes) return RIGA_ERR_INVALID_ARG;
  *out = nullptr;
  riga_batch* bh = new (std::nothrow) riga_batch();
  if (!bh) return RIGA_ERR_OOM;
  bh->n = n;
  bh->device = device;
  bh->user_st = (hipStream_t)hip_stream;
  bh->meshes.assign(meshes, meshes + n);
  bh->plans.resize(n);
  std::vector<int> bad(n, 0);
  parallel_for(n, [&](int i) {
    bad[i] = meshes[i].space != RIGA_SPACE_H1
                 ? -1
                 : bh->plans[i].build(meshes[i].p, meshes[i].ne, meshes[i].hyper_every, meshes[i].leaf);
    if (bad[i] == 0) bh->plans[i].ensure_symbolic();   // algorithmic factor flops of the forest
  });
  for (int i = 0; i < n; ++i)
    if (bad[i] != 0) {
      delete bh;
      return RIGA_ERR_INVALID_ARG;
    }
  riga_status rc = run([&]() -> riga_status {
    ck(hipSetDevice(device));
    riga_problem* fp = new riga_problem();
    bh->fp = fp;
    std::vector<const riga::Plan*> parts(n);
    for (int i = 0; i < n; ++i) parts[i] = &bh->plans[i];
    fp->plan.merge(parts, bh->dof_base, bh->node_base);
    fp->device = device;
    fp->st = bh->user_st;
    fp->mesh = riga_mesh{0, 0, 0, 0};
    fp->node_inst.assign(fp->plan.nodes.size(), 0);
    for (int i = 0; i < n; ++i)
      for (int v = bh->node_base[i]; v < bh->node_base[i + 1]; ++v) fp->node_inst[v] = i;
    setup_device(fp);
    {
      std::vector<int4> ranges(n);
      for (int i = 0; i < n; ++i) ranges[i] = int4{i, (int)bh->dof_base[i], (int)bh->dof_base[i + 1], 0};
      setup_ell(fp, ranges);
    }
    const int64_t T = fp->plan.ndof;
    // per-problem 1-D spaces in shared arrays, rows into the forest CSR
    std::vector<int> knots, sup0, sup1, lo, hi, first;
    struct Off { size_t kn, sp, el; };
    std::vector<Off> off(n);
    for (int i = 0; i < n; ++i) {
      const riga::Space1D& S = bh->plans[i].sp;
      off[i] = {knots.size(), sup0.size(), first.size()};
      knots.insert(knots.end(), S.knots.begin(), S.knots.end());
      sup0.insert(sup0.end(), S.sup0.begin(), S.sup0.end());
      sup1.insert(sup1.end(), S.sup1.begin(), S.sup1.end());
      lo.insert(lo.end(), S.lo.begin(), S.lo.end());
      hi.insert(hi.end(), S.hi.begin(), S.hi.end());
      first.insert(first.end(), S.first.begin(), S.first.end());
    }
    const int* dk = fp->upload(knots);
    const int *d0 = fp->upload(sup0), *d1 = fp->upload(sup1), *dlo = fp->upload(lo), *dhi = fp->upload(hi);
    const int* dfi = fp->upload(first);
    bh->hsp.resize(n);
    size_t tab = 0;
    std::vector<size_t> taboff(n);
    for (int i = 0; i < n; ++i) {
      const riga::Space1D& S = bh->plans[i].sp;
      riga::DevSpace& d = bh->hsp[i];
      d.p = S.p; d.ne = S.ne; d.n = S.n;
      d.knots = dk + off[i].kn;
      d.sup0 = d0 + off[i].sp; d.sup1 = d1 + off[i].sp;
      d.lo = dlo + off[i].sp; d.hi = dhi + off[i].sp;
      d.first = dfi + off[i].el;
      d.rowptr = fp->ds.rowptr + bh->dof_base[i];
      taboff[i] = tab;
      tab += (size_t)S.ne * (S.p + 1) * (S.p + 1);
    }
    double* dtM = fp->dalloc<double>(tab);
    double* dtK = fp->dalloc<double>(tab);
    bh->tabM.resize(n); bh->tabK.resize(n); bh->gx.resize(n); bh->gw.resize(n);
    std::map<int, std::pair<double*, double*>> rule;
    for (int i = 0; i < n; ++i) {
      bh->tabM[i] = dtM + taboff[i];
      bh->tabK[i] = dtK + taboff[i];
      const int p = bh->plans[i].sp.p;
      if (!rule.count(p)) {
        std::vector<double> x, w;
        gauss_legendre(p + 1, x, w);
        rule[p] = {fp->upload(x), fp->upload(w)};
      }
      bh->gx[i] = rule[p].first;
      bh->gw[i] = rule[p].second;
    }
    // per-problem tables of the batched assembly
    {
      std::vector<int64_t> to(n);
      for (int i = 0; i < n; ++i) {
        to[i] = (int64_t)taboff[i];
        bh->max_ne = std::max(bh->max_ne, bh->plans[i].sp.ne);
      }
      bh->d_taboff = fp->upload(to);
      bh->d_gx = fp->upload(std::vector<const double*>(bh->gx.begin(), bh->gx.end()));
      bh->d_gw = fp->upload(std::vector<const double*>(bh->gw.begin(), bh->gw.end()));
      bh->d_tabM = dtM;
      bh->d_tabK = dtK;
      bh->d_alpha = fp->dalloc<double>(n);
      bh->d_beta = fp->dalloc<double>(n);
      bh->d_celem = fp->dalloc<const double*>(n);
    }
    // problem of every node and row; row blocks and dot blocks
    std::vector<int> rinst(T);
    std::vector<int4> rb, db;
    std::vector<int> dboff(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      const int64_t r0 = bh->dof_base[i], r1 = bh->dof_base[i + 1];
      for (int64_t r = r0; r < r1; ++r) rinst[r] = i;
      for (int64_t r = r0; r < r1; r += 256) rb.push_back(int4{i, (int)r, (int)std::min(r + 256, r1), 0});
      for (int64_t r = r0; r < r1; r += DOT_ROWS) db.push_back(int4{i, (int)r, (int)std::min(r + DOT_ROWS, r1), 0});
      dboff[i + 1] = (int)db.size();
    }
    riga::BatchDev& B = bh->B;
    B.n = n;
    B.ntot = T;
    B.rinst = fp->upload(rinst);
    B.spaces = fp->upload(bh->hsp);
    B.dofbase = fp->upload(bh->dof_base);
    B.sig = fp->dalloc<double>(n);
    B.live = fp->dalloc<unsigned char>(n);
    B.kcur = fp->dalloc<int>(n);
    B.flag = fp->dalloc<int>(n);
    B.rb = fp->upload(rb);
    bh->rb_problem.resize(rb.size());
    for (size_t b = 0; b < rb.size(); ++b) bh->rb_problem[b] = rb[b].x;
    B.nrb = (int)rb.size();
    B.db = fp->upload(db);
    B.ndb = (int)db.size();
    B.dboff = fp->upload(dboff);
    std::vector<int64_t> nzb(n + 1);
    for (int i = 0; i <= n; ++i) nzb[i] = fp->plan.rowptr[bh->dof_base[i]];
    bh->d_nzbase = fp->upload(nzb);
    {
      std::vector<int4> tiles;
      std::vector<int64_t> bo(n);
      int64_t boff = 0;
      for (int i = 0; i < n; ++i) {
        const riga::Space1D& S = bh->plans[i].sp;
        bo[i] = boff;
        boff += (int64_t)S.n * (2 * S.p + 1);
        bh->max_p = std::max(bh->max_p, S.p);
        bh->max_w = std::max(bh->max_w, S.n * (2 * S.p + 1));
        for (int j0 = 0; j0 < S.n; j0 += riga::TENSOR_TILE_J)
          for (int i0 = 0; i0 < S.n; i0 += riga::TENSOR_TILE_I) tiles.push_back(int4{i, i0, j0, 0});
      }
      bh->d_ttiles = fp->upload(tiles);
      bh->nttiles = (int)tiles.size();
      bh->d_bandoff = fp->upload(bo);
      bh->d_M1 = fp->dalloc<double>((size_t)boff);
      bh->d_K1 = fp->dalloc<double>((size_t)boff);
    }
    fp->dt.inst = fp->upload(fp->node_inst);
    fp->dt.spaces = B.spaces;
    fp->dt.dofbase = B.dofbase;
    fp->dt.isig = B.sig;
    return RIGA_OK;
  });
  if (rc != RIGA_OK) {
    riga_batch_destroy(bh);
    return rc;
  }
  *out = bh;
  return RIGA_OK;
}

void riga_batch_destroy(riga_batch* bh) {
  if (!bh) return;
  if (bh->fp) {
    hipSetDevice(bh->device);
    if (bh->fp->own_st) hipStreamSynchronize(bh->fp->own_st);
    bh->clear_graphs();
    riga_destroy(bh->fp);
  }
  delete bh;
}

riga_status riga_batch_info(const riga_batch* bh, int64_t* total_dofs, int64_t* dof_offsets) {
  if (!bh) return RIGA_ERR_INVALID_ARG;
  if (total_dofs) *total_dofs = bh->dof_base[bh->n];
  if (dof_offsets) std::memcpy(dof_offsets, bh->dof_base.data(), (bh->n + 1) * sizeof(int64_t));
  return RIGA_OK;
}

riga_status riga_batch_assemble(riga_batch* bh, const riga_damping* damping) {
  if (!bh || !damping) return RIGA_ERR_INVALID_ARG;
  return run([&]() -> riga_status {
    ck(hipSetDevice(bh->device));
    riga_problem* fp = bh->fp;
    const int n = bh->n;
    hipStream_t st = bh->user_st;
    ck(hipEventRecord(fp->ev0, st));
    bh->clear_graphs();   // captured block steps hold the old operator coefficients
    bh->alpha.resize(n); bh->beta.resize(n); bh->celem.resize(n);
    for (int i = 0; i < n; ++i) {
      bh->alpha[i] = damping[i].alpha; bh->beta[i] = damping[i].beta; bh->celem[i] = damping[i].c_elem;
    }
    // the damping of every problem, then tables, bands and entries of all problems in three launches
    ck(hipMemcpyAsync(bh->d_alpha, bh->alpha.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    ck(hipMemcpyAsync(bh->d_beta, bh->beta.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    ck(hipMemcpyAsync((void*)bh->d_celem, bh->celem.data(), n * sizeof(const double*), hipMemcpyHostToDevice, st));
    riga::launch_assemble_b(bh->B.rb, bh->B.nrb, bh->B.spaces, bh->B.dofbase, bh->d_taboff, bh->d_gx, bh->d_gw, n,
                            bh->max_ne, bh->d_tabM, bh->d_tabK, bh->max_w, bh->d_bandoff, bh->d_M1, bh->d_K1,
                            bh->d_alpha, bh->d_beta, bh->d_celem, fp->d_K, fp->d_M, fp->d_C, st);
    bh->any_field = false;
    for (int i = 0; i < n; ++i) bh->any_field = bh->any_field || bh->celem[i] != nullptr;
    ck(hipEventRecord(fp->ev1, st));
    // 1-norms per problem (largest absolute row sums): one launch over the row
    // blocks of the forest, one synchronisation
    const int nrb = bh->B.nrb;
    double* part = fp->d_part;   // 512 * 400 * 4 doubles: room for 3 per row block up to 273,066 blocks
    if ((size_t)nrb * 3 > (size_t)512 * 400 * 4) throw std::bad_alloc();
    riga::launch_rowabs3(bh->B.rb, nrb, fp->N(), 0, fp->ds.rowptr, fp->d_K, fp->d_C, fp->d_M, part, st);
    std::vector<double> h((size_t)nrb * 3);
    ck(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ck(hipStreamSynchronize(st));
    bh->norms.assign((size_t)n * 3, 0.0);
    for (int b = 0; b < nrb; ++b)
      for (int a = 0; a < 3; ++a) {
        double& v = bh->norms[(size_t)bh->rb_problem[b] * 3 + a];
        v = std::max(v, h[(size_t)b * 3 + a]);
      }
    float ms = 0;
    ck(hipEventElapsedTime(&ms, fp->ev0, fp->ev1));
    bh->stats.t_assemble_ms = ms;
    bh->assembled = true;
    bh->factored = false;
    fp->assembled = true;
    return RIGA_OK;
  });
}

riga_status riga_batch_factor(riga_batch* bh, const double* sigmas, int64_t* bad_pivot) {
  if (!bh || !sigmas) return RIGA_ERR_INVALID_ARG;
  for (int i = 0; i < bh->n; ++i)
    if (!(sigmas[i] > 0.0) || !std::isfinite(sigmas[i])) return RIGA_ERR_INVALID_ARG;
  if (bad_pivot)
    for (int i = 0; i < bh->n; ++i) bad_pivot[i] = -1;
  if (!bh->assembled) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(bh->device));
    riga_problem* fp = bh->fp;
    bh->sigma.assign(sigmas, sigmas + bh->n);
    ck(hipMemcpyAsync((void*)bh->B.sig, sigmas, bh->n * sizeof(double), hipMemcpyHostToDevice, bh->user_st));
    fp->dt.ilive = nullptr;
    int64_t bad = -1;
    riga_status rc = factor_all(fp, 1.0, &bad);
    riga::launch_combine_b(bh->n, bh->d_nzbase, fp->plan.nnz, bh->B.sig, fp->d_M, fp->d_C, fp->d_A, bh->user_st);
    // the operator's sparse copy is needed only with an element damping field
    if (bh->any_field)
      riga::launch_csr_to_ell(fp->d_slabs, fp->nslab, fp->ds.rowptr, fp->d_A, fp->d_Aell, bh->user_st);
    bh->stats.t_factor_ms = fp->stats.t_factor_ms;
    if (rc == RIGA_ERR_NOT_SPD && bad >= 0) {
      const int i = (int)(std::upper_bound(bh->dof_base.begin(), bh->dof_base.end(), bad) - bh->dof_base.begin()) - 1;
      if (bad_pivot && i >= 0 && i < bh->n) bad_pivot[i] = bad - bh->dof_base[i];
    }
    bh->factored = rc == RIGA_OK;
    bh->clear_graphs();
    return rc;
  });
}

riga_status riga_batch_eigs(riga_batch* bh, const riga_options* opt, double* lam, double* X, double* eta,
                            int* nconv) {
  if (!bh || !opt || !lam || !nconv || opt->v0) return RIGA_ERR_INVALID_ARG;
  if (!bh->factored) return RIGA_ERR_STATE;
  const int n = bh->n;
  const int nev = opt->nev;
  const int b = opt->block > 0 ? opt->block : 2;
  const int m = opt->m > 0 ? opt->m : std::max(2 * nev, 20);
  const int maxit = opt->maxit > 0 ? opt->maxit : 200;
  const double tol = opt->tol > 0 ? opt->tol : 1e-12;
  if (nev < 1 || b < 1 || b > 4 || m < nev + b || m + 2 * b > 256 || opt->keep < 0 || opt->keep > m - b)
    return RIGA_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (2 * bh->N(i) < m) return RIGA_ERR_INVALID_ARG;
  riga_problem* fp = bh->fp;
  return run([&]() -> riga_status {
    ck(hipSetDevice(bh->device));
    hipStream_t st = fp->own_st;
    ck(hipEventRecord(fp->ev_fence, bh->user_st));
    ck(hipStreamWaitEvent(st, fp->ev_fence, 0));
    const int ldh = m + 2 * b;
    ensure_workspace(bh, ldh, b);
    if (bh->graph_b != b || bh->graph_m != m) {
      bh->clear_graphs();
      bh->graph_b = b;
      bh->graph_m = m;
    }
    riga::BatchDev& B = bh->B;
    const int64_t T = B.ntot;
    hipStream_t save_st = fp->st;
    fp->st = st;   // the sweeps run on the batch's stream
    struct Restore {
      riga_problem* fp; hipStream_t s;
      ~Restore() { fp->st = s; fp->dt.ilive = nullptr; }
    } restore{fp, save_st};
    ck(hipEventRecord(fp->ev0, st));
    // --- start block: random, B-orthonormalised per problem -------------------
    std::vector<unsigned char> live(n, 1);
    std::vector<int> kc(n, 0);
    ck(hipMemcpyAsync(B.live, live.data(), n, hipMemcpyHostToDevice, st));
    ck(hipMemcpyAsync(B.kcur, kc.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    ck(hipMemsetAsync(B.flag, 0, n * sizeof(int), st));
    ck(hipMemsetAsync(bh->H, 0, sizeof(double) * (size_t)n * ldh * ldh, st));
    riga::launch_random_fill(bh->Ru, T, b, T, opt->seed * 2 + 1, st);
    riga::launch_random_fill(bh->Rl, T, b, T, opt->seed * 2 + 2, st);
    riga::launch_tensor_mk_b(bh->d_ttiles, bh->nttiles, B.spaces, B.dofbase, bh->d_bandoff, bh->d_M1, bh->d_K1,
                             B.live, nullptr, nullptr, nullptr, b, bh->max_p, bh->Rl, T, bh->MRl, T, nullptr, 0, 0.0,
                             st);
    riga::launch_dots_b(B, 0, b, false, bh->Ru, bh->MRl, b, bh->Ru, bh->Rl, bh->G, b * b, st);
    riga::launch_block_normalize_b(B, false, 0, b, nullptr, nullptr, 0, bh->G, nullptr, ldh, bh->Rinv, st);
    riga::launch_gemm3_b(B, false, 0, b, bh->Rinv, bh->Ru, bh->Vu, bh->Rl, bh->Vl, bh->MRl, bh->Wl, st);
    fp->dt.ilive = B.live;
    // --- lockstep cycles ----------------------------------------------------------
    enum { ACTIVE = 0, CONVERGED = 1, MAXIT = 2, BROKE = 3 };
    std::vector<int> state(n, ACTIVE), it(n, 0), kend(n, 0);
    std::vector<riga::KsCycle> cyc(n);
    const size_t hl = (size_t)ldh * ldh;
    // host staging in pinned memory (every copy a direct asynchronous one):
    // down: projected matrices and breakdown flags; up: per problem a slot of
    // 2 ldh^2 combination coefficients, the new projected matrices and the
    // small per-problem arrays
    const size_t nh = (size_t)n * hl, nq2 = (size_t)n * 2 * hl;
    double* const pin = fp->pinned(nh + n + nq2 + nh + 5 * (size_t)n + 8);
    double* const dnH = pin;
    const int* const dnFlag = reinterpret_cast<const int*>(pin + nh);
    double* const Qh = pin + nh + n;
    double* const Hh = Qh + nq2;
    int* const hkin = reinterpret_cast<int*>(Hh + nh);   // n ints in n / 2 doubles
    int* const hkout = hkin + n;
    int64_t* const hqoff = reinterpret_cast<int64_t*>(Hh + nh + n);
    int* const hkc = reinterpret_cast<int*>(Hh + nh + 2 * (size_t)n);
    unsigned char* const hlive = reinterpret_cast<unsigned char*>(Hh + nh + 3 * (size_t)n);
    int* const hkin_f = reinterpret_cast<int*>(Hh + nh + 4 * (size_t)n);   // n ints each
    int* const hkout_f = hkin_f + n;
    int64_t n_fb = 0;
    int cycles = 0;
    double t_host = 0.0;
    for (;;) {
      int steps = 0;
      for (int i = 0; i < n; ++i)
        if (state[i] == ACTIVE) steps = std::max(steps, (m - kc[i]) / b);
      for (int s = 0; s < steps; ++s) {
        if (opt->flags & 1) {
          enqueue_step(bh, b, m, ldh, st);
        } else {
          auto git = bh->graphs.find(bh->Vu);
          if (git == bh->graphs.end()) {
            ck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            enqueue_step(bh, b, m, ldh, st);
            hipGraph_t g = nullptr;
            ck(hipStreamEndCapture(st, &g));
            hipGraphExec_t ex = nullptr;
            hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            ck(e);
            git = bh->graphs.emplace(bh->Vu, ex).first;
          }
          ck(hipGraphLaunch(git->second, st));
        }
      }
      ++cycles;
      // projected matrices and breakdown flags of every problem
      ck(hipMemcpyAsync(dnH, bh->H, sizeof(double) * nh, hipMemcpyDeviceToHost, st));
      ck(hipMemcpyAsync((void*)dnFlag, B.flag, sizeof(int) * n, hipMemcpyDeviceToHost, st));
      ck(hipStreamSynchronize(st));
      const auto th0 = std::chrono::steady_clock::now();   // the device waits from here
      std::vector<int> newstate(state);
      parallel_for(n, [&](int i) {
        if (state[i] != ACTIVE) return;
        const int steps_i = (m - kc[i]) / b;
        const int k = kc[i] + steps_i * b;
        kend[i] = k;
        if (dnFlag[i]) { newstate[i] = BROKE; return; }
        std::vector<double> Hi(dnH + (size_t)i * hl, dnH + (size_t)(i + 1) * hl);
        if (riga::ks_ritz(Hi, ldh, k, b, nev, tol, cyc[i]) != 0) { newstate[i] = BROKE; return; }
        ++it[i];
        if (cyc[i].nconv == cyc[i].nw) { newstate[i] = CONVERGED; return; }
        if (it[i] >= maxit) { newstate[i] = MAXIT; return; }
        riga::ks_restart(Hi, ldh, k, b, m, nev, opt->keep, cyc[i]);
      });
      for (int i = 0; i < n; ++i)
        if (state[i] == ACTIVE) n_fb += (int64_t)b * ((m - kc[i]) / b);
      // finished problems: Ritz vectors u = V_u y (planar [Re | Im]) before the restart
      std::vector<int> fin, rst;
      for (int i = 0; i < n; ++i) {
        if (state[i] != ACTIVE) continue;
        if (newstate[i] == CONVERGED || newstate[i] == MAXIT) fin.push_back(i);
        else if (newstate[i] == ACTIVE) rst.push_back(i);
      }
      // Finished problems' Ritz vectors and the others' restart combinations go to
      // disjoint per-problem slots of one staging area and one upload; the
      // problems' products are queued (Ritz vectors first: they read the basis
      // the restart replaces) and the next cycle follows them in stream order.
      // The staging area is rewritten only after the next cycle's download has
      // been waited for, so no wait is needed here.
      std::fill(hkout_f, hkout_f + n, 0);
      std::fill(hkout, hkout + n, 0);
      std::fill(Hh, Hh + nh, 0.0);
      int max_kin_f = 1, max_kout_f = 1, max_kin = 1, max_kout = 1;
      for (int i = 0; i < n; ++i) hqoff[i] = (int64_t)i * 2 * hl;
      for (int i : fin) {
        const int k = kend[i], nw = cyc[i].nw;
        riga::ks_ritz_vectors(cyc[i]);
        double* q = Qh + (size_t)i * 2 * hl;
        for (int j = 0; j < nw; ++j)
          for (int c = 0; c < k; ++c) {
            const cplx y = cyc[i].Y[c + (size_t)cyc[i].wanted[j] * k];
            q[c + (size_t)j * k] = y.real();
            q[c + (size_t)(nw + j) * k] = y.imag();
          }
        hkin_f[i] = k; hkout_f[i] = 2 * nw;
        max_kin_f = std::max(max_kin_f, k);
        max_kout_f = std::max(max_kout_f, 2 * nw);
      }
      state = newstate;
      // restart: V_new = [V_k Qk, V_{k:k+b}] per problem, new H, k = r
      for (int i : rst) {
        const riga::KsCycle& c = cyc[i];
        const int kin = kend[i] + b, kout = c.r + b;
        std::memcpy(Qh + (size_t)i * 2 * hl, c.Qe.data(), c.Qe.size() * sizeof(double));
        hkin[i] = kin; hkout[i] = kout;
        max_kin = std::max(max_kin, kin);
        max_kout = std::max(max_kout, kout);
        std::memcpy(Hh + (size_t)i * hl, c.Hn.data(), hl * sizeof(double));
        kc[i] = c.r;
      }
      for (int i = 0; i < n; ++i) live[i] = state[i] == ACTIVE ? 1 : 0;
      std::memcpy(hkc, kc.data(), sizeof(int) * n);
      std::memcpy(hlive, live.data(), n);
      t_host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
      ck(hipMemcpyAsync(bh->Qd, Qh, sizeof(double) * nq2, hipMemcpyHostToDevice, st));
      ck(hipMemcpyAsync(bh->qoff, hqoff, sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
      if (!fin.empty()) {
        ck(hipMemcpyAsync(bh->kin_f, hkin_f, sizeof(int) * n, hipMemcpyHostToDevice, st));
        ck(hipMemcpyAsync(bh->kout_f, hkout_f, sizeof(int) * n, hipMemcpyHostToDevice, st));
        riga::launch_gemm_tall_b(B, bh->kin_f, bh->kout_f, bh->qoff, bh->Qd, max_kin_f, max_kout_f, bh->Vu, bh->P, st);
      }
      if (rst.empty()) break;
      ck(hipMemcpyAsync(bh->kin, hkin, sizeof(int) * n, hipMemcpyHostToDevice, st));
      ck(hipMemcpyAsync(bh->kout, hkout, sizeof(int) * n, hipMemcpyHostToDevice, st));
      riga::launch_gemm_tall_b(B, bh->kin, bh->kout, bh->qoff, bh->Qd, max_kin, max_kout, bh->Vu, bh->Vu2, st);
      riga::launch_gemm_tall_b(B, bh->kin, bh->kout, bh->qoff, bh->Qd, max_kin, max_kout, bh->Vl, bh->Vl2, st);
      riga::launch_gemm_tall_b(B, bh->kin, bh->kout, bh->qoff, bh->Qd, max_kin, max_kout, bh->Wl, bh->Wl2, st);
      std::swap(bh->Vu, bh->Vu2); std::swap(bh->Vl, bh->Vl2); std::swap(bh->Wl, bh->Wl2);
      ck(hipMemcpyAsync(bh->H, Hh, sizeof(double) * nh, hipMemcpyHostToDevice, st));
      ck(hipMemcpyAsync(B.kcur, hkc, sizeof(int) * n, hipMemcpyHostToDevice, st));
      ck(hipMemcpyAsync(B.live, hlive, n, hipMemcpyHostToDevice, st));
    }
    fp->dt.ilive = nullptr;
    // --- eigenpairs of every finished problem ------------------------------------
    std::vector<int> done;
    for (int i = 0; i < n; ++i)
      if (state[i] == CONVERGED || state[i] == MAXIT) done.push_back(i);
    const int nsplit = 8;
    const size_t pst = (size_t)2 * ldh * nsplit * 11;   // part stride per problem
    for (int i : done) {
      const int nw = cyc[i].nw;
      const int64_t o = bh->dof_base[i];
      const int64_t Ni = bh->N(i);
      for (int c0 = 0; c0 < 2 * nw; c0 += 8) {
        const int nc = std::min(8, 2 * nw - c0);
        const double* x = bh->P + (size_t)c0 * T + o;
        riga::launch_spmv3(bh->hsp[i], Ni, nc, fp->d_M, fp->d_C, fp->d_K, x, T, bh->MP + (size_t)c0 * T + o,
                           bh->CP + (size_t)c0 * T + o, bh->KP + (size_t)c0 * T + o, T, st);
      }
      riga::launch_pair_forms(Ni, nw, bh->P + o, bh->MP + o, bh->CP + o, bh->KP + o, T, bh->part + (size_t)i * pst,
                              nsplit, st);
    }
    std::vector<double> parts((size_t)n * pst);
    ck(hipMemcpyAsync(parts.data(), bh->part, parts.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ck(hipStreamSynchronize(st));
    std::vector<std::vector<cplx>> lrq(n);
    std::vector<std::vector<double>> uMu(n), un2(n);
    std::vector<double> lamd((size_t)n * 2 * ldh, 0.0);
    for (int i : done) {
      const int nw = cyc[i].nw;
      lrq[i].resize(nw); uMu[i].resize(nw); un2[i].resize(nw);
      for (int j = 0; j < nw; ++j) {
        double f[11] = {0};
        for (int x = 0; x < nsplit; ++x)
          for (int t2 = 0; t2 < 11; ++t2) f[t2] += parts[(size_t)i * pst + ((size_t)j * nsplit + x) * 11 + t2];
        const riga::PairForms pf = riga::pair_forms(f);
        uMu[i][j] = pf.uMu;
        un2[i][j] = pf.unorm2;
        lrq[i][j] = riga::rayleigh_polish(pf, bh->sigma[i] + 1.0 / cyc[i].theta[cyc[i].wanted[j]]);
        lamd[(size_t)i * 2 * ldh + 2 * j] = lrq[i][j].real();
        lamd[(size_t)i * 2 * ldh + 2 * j + 1] = lrq[i][j].imag();
      }
    }
    ck(hipMemcpyAsync(bh->dlam, lamd.data(), lamd.size() * sizeof(double), hipMemcpyHostToDevice, st));
    for (int i : done) {
      const int64_t o = bh->dof_base[i];
      riga::launch_pair_resid(bh->N(i), cyc[i].nw, bh->P + o, bh->MP + o, bh->CP + o, bh->KP + o, T,
                              bh->dlam + (size_t)i * 2 * ldh, bh->part + (size_t)i * pst, nsplit, st);
    }
    ck(hipMemcpyAsync(parts.data(), bh->part, parts.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ck(hipStreamSynchronize(st));
    std::vector<double> sc((size_t)n * 3 * nev, 0.0);
    bool all_conv = true;
    for (int i = 0; i < n; ++i) {
      nconv[i] = 0;
      for (int j = 0; j < nev; ++j) {
        lam[(size_t)i * 2 * nev + 2 * j] = NAN;
        lam[(size_t)i * 2 * nev + 2 * j + 1] = NAN;
        if (eta) eta[(size_t)i * nev + j] = NAN;
      }
      if (state[i] != CONVERGED) all_conv = false;
    }
    for (int i : done) {
      const int nw = cyc[i].nw;
      std::vector<double> etav(nw);
      std::vector<cplx> umax(nw);
      for (int j = 0; j < nw; ++j) {
        double s = 0.0, best = -1.0;
        for (int x = 0; x < nsplit; ++x) {
          const double* o = &parts[(size_t)i * pst + ((size_t)j * nsplit + x) * 5];
          s += o[0];
          if (o[1] > best) { best = o[1]; umax[j] = cplx(o[3], o[4]); }
        }
        etav[j] = riga::scaled_residual(s, lrq[i][j], &bh->norms[(size_t)i * 3], un2[i][j]);
      }
      std::vector<int> order = canonical_order(lrq[i], bh->sigma[i]);
      const int nout = std::min(nev, nw);
      // leading pairs in canonical order whose explicit residual meets the bar
      int cnt = 0;
      for (int j = 0; j < nout; ++j) {
        if (etav[order[j]] <= riga::detail::kEtaConverged) ++cnt; else break;
      }
      if (cnt < nev) all_conv = false;
      nconv[i] = cnt;
      for (int j = 0; j < nout; ++j) {
        lam[(size_t)i * 2 * nev + 2 * j] = lrq[i][order[j]].real();
        lam[(size_t)i * 2 * nev + 2 * j + 1] = lrq[i][order[j]].imag();
        if (eta) eta[(size_t)i * nev + j] = etav[order[j]];
        const int src = order[j];
        const cplx ph = std::conj(umax[src]) / std::abs(umax[src]);
        const cplx s = ph / std::sqrt(uMu[i][src]);
        sc[((size_t)i * nev + j) * 3] = s.real();
        sc[((size_t)i * nev + j) * 3 + 1] = s.imag();
        sc[((size_t)i * nev + j) * 3 + 2] = (double)src;
      }
    }
    if (X) {
      double* dsc = bh->Qd;   // free again: scale factors of every problem
      ck(hipMemcpyAsync(dsc, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, st));
      for (int i : done) {
        const int64_t o = bh->dof_base[i];
        riga::launch_finalize(bh->N(i), cyc[i].nw, std::min(nev, cyc[i].nw), bh->P + o, T,
                              dsc + (size_t)i * 3 * nev, X + 2 * (size_t)nev * o, st);
      }
    }
    ck(hipEventRecord(fp->ev1, st));
    ck(hipStreamSynchronize(st));
    float ms = 0;
    ck(hipEventElapsedTime(&ms, fp->ev0, fp->ev1));
    bh->stats.t_eigs_ms = ms;
    bh->stats.n_it = cycles;
    bh->stats.n_fb = n_fb;
    bh->stats.n_mv = 3 * n_fb;
    bh->stats.n_vv = 0;
    bh->stats.n_ir = 0;
    bh->stats.t_host_ms = t_host;
    // problems whose block lost rank are solved again one by one on the
    // host-checked path of the single-problem driver
    for (int i = 0; i < n; ++i) {
      if (state[i] != BROKE) continue;
      riga_problem* sp = nullptr;
      riga_mesh me = bh->meshes[i];
      if (riga_create(&sp, &me, bh->device, (void*)st) != RIGA_OK) throw HipError{hipErrorUnknown};
      riga_damping dm{bh->alpha[i], bh->beta[i], bh->celem[i]};
      riga_options o2 = *opt;
      o2.flags |= 2;
      o2.m = m;
      int nc1 = 0;
      std::vector<double> l1(2 * nev), e1(nev);
      riga_status r1 = riga_assemble(sp, &dm);
      if (r1 == RIGA_OK) r1 = riga_factor(sp, bh->sigma[i], nullptr);
      if (r1 == RIGA_OK)
        r1 = riga_eigs(sp, &o2, l1.data(), X ? X + 2 * (size_t)nev * bh->dof_base[i] : nullptr, e1.data(), &nc1);
      riga_destroy(sp);
      if (r1 < 0) return r1;
      nconv[i] = nc1;
      for (int j = 0; j < nev; ++j) {
        lam[(size_t)i * 2 * nev + 2 * j] = l1[2 * j];
        lam[(size_t)i * 2 * nev + 2 * j + 1] = l1[2 * j + 1];
        if (eta) eta[(size_t)i * nev + j] = e1[j];
      }
    }
    bh->n_broke = 0;
    for (int i = 0; i < n; ++i) bh->n_broke += state[i] == BROKE;
    all_conv = true;
    for (int i = 0; i < n; ++i)
      if (nconv[i] < nev) all_conv = false;
    return all_conv ? RIGA_OK : RIGA_WARN_NOT_CONVERGED;
  });
}

riga_status riga_batch_autotune(riga_batch* bh, int nrhs, int reps, double* before_ms, double* after_ms) {
  if (!bh || nrhs < 1 || nrhs > 4 || reps < 1) return RIGA_ERR_INVALID_ARG;
  if (!bh->factored) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(bh->device));
    bh->fp->dt.ilive = nullptr;
    autotune_sweeps(bh->fp, nrhs, reps, before_ms, after_ms);
    bh->clear_graphs();
    return RIGA_OK;
  });
}

riga_status riga_batch_stats(const riga_batch* bh, riga_stats_t* stats, int* n_resolved) {
  if (!bh || !stats) return RIGA_ERR_INVALID_ARG;
  *stats = bh->stats;
  if (n_resolved) *n_resolved = bh->n_broke;
  return RIGA_OK;
}

}  // extern "C"
