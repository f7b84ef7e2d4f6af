// Host-only checks of the library's plain C++ parts, built by
// tests/test_host_sanitizers.py with the address + undefined-behaviour
// sanitizers ("asan") or the thread sanitizer ("tsan"):
//   - the nested-dissection plan (Sec. 3.3 hyperplanes as separators), its
//     symbolic Cholesky and the forest merge of the batched form; the
//     curl-conforming plan and the real form of a complex system;
//   - the dense real Schur form of a projected matrix (eq. ArnoldiRitz) and
//     the reordering of the Krylov--Schur restart (Sec. 4.1.3);
//   - the symmetric Jacobi eigensolver of the Lanczos slices (Sec. 4.1.2);
//   - one Rayleigh--Ritz + restart cycle on a random block Hessenberg matrix;
//   - the host worker pool, including a job that throws.
// Exit status 0 when every check passes; a sanitizer report fails the run.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <stdexcept>
#include <vector>

#include "host_pool.hpp"
#include "ks_host.hpp"
#include "plan.hpp"
#include "small_eig.hpp"

namespace {

int failures = 0;
void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

void plans() {
  const int meshes[][4] = {{2, 16, 4, 0}, {3, 24, 8, 0}, {3, 20, 0, 4}, {4, 16, 8, 2}, {1, 8, 0, 0}, {5, 12, 6, 0}};
  std::vector<riga::Plan> ps(sizeof(meshes) / sizeof(meshes[0]));
  for (size_t k = 0; k < ps.size(); ++k) {
    const int* m = meshes[k];
    check(ps[k].build(m[0], m[1], m[2], m[3]) == 0, "plan build");
    const riga::Plan& P = ps[k];
    std::vector<char> seen(P.ndof, 0);
    for (int64_t d = 0; d < P.ndof; ++d) {
      const int64_t e = P.elim_pos[d];
      check(e >= 0 && e < P.ndof && !seen[e], "elimination order is a permutation");
      if (e >= 0 && e < P.ndof) seen[e] = 1;
    }
    std::vector<int64_t> cc;
    int64_t nz = 0;
    double fl = 0.0;
    P.symbolic(&cc, nz, fl);
    int64_t sum = 0;
    for (int64_t c : cc) {
      check(c >= 1, "column count includes the diagonal");
      sum += c;
    }
    check(sum == nz && fl >= 0.0, "symbolic totals");
    ps[k].ensure_symbolic();
  }
  check(riga::Plan().build(0, 8, 0, 0) < 0, "degree 0 rejected");
  check(riga::Plan().build(2, 10, 3, 0) < 0, "spacing must divide the mesh");
  std::vector<const riga::Plan*> parts;
  for (auto& p : ps) parts.push_back(&p);
  riga::Plan F;
  std::vector<int64_t> db;
  std::vector<int> nbase;
  F.merge(parts, db, nbase);
  int64_t tot = 0, nzs = 0;
  for (auto& p : ps) {
    tot += p.ndof;
    nzs += p.sym_nnz_l;
  }
  check(F.ndof == tot && db.back() == tot, "forest dofs");
  check(F.sym_nnz_l == nzs, "forest symbolic total");
}

// The curl-conforming plan (explicit columns) and the real form of a complex
// system on a plan (two unknowns per dof): every coupling a full 2 x 2 block,
// the same tree with fronts exactly twice as large, a dof's two unknowns
// eliminated at the same node.
void realform_plans() {
  riga::Plan bases[3];
  check(bases[0].build(2, 16, 4, 0) == 0, "scalar plan");
  check(bases[1].build(3, 24, 0, 8) == 0, "scalar IGA plan");
  check(bases[2].build_hcurl(3, 16, 8, 0, true) == 0, "curl-conforming plan");
  for (const riga::Plan& b : bases) {
    riga::Plan r;
    check(r.build_realform(b) == 0, "real-form plan");
    check(r.ndof == 2 * b.ndof && r.nnz == 4 * b.nnz, "real-form sizes");
    check(r.nodes.size() == b.nodes.size(), "real-form tree");
    for (size_t v = 0; v < b.nodes.size() && v < r.nodes.size(); ++v)
      check(r.no[v] == 2 * b.no[v] && r.nb[v] == 2 * b.nb[v], "real-form fronts");
    for (int64_t d = 0; d < b.ndof; ++d) {
      check(r.node_of_dof[2 * d] == r.node_of_dof[2 * d + 1], "unknowns of a dof together");
      const int64_t len = b.rowptr[d + 1] - b.rowptr[d];
      check(r.rowptr[2 * d] == 4 * b.rowptr[d] && r.rowptr[2 * d + 1] - r.rowptr[2 * d] == 2 * len,
            "real-form rows");
    }
    for (int64_t i = 0; i < r.ndof; ++i)
      for (int64_t q = r.rowptr[i] + 1; q < r.rowptr[i + 1]; ++q) check(r.col[q] > r.col[q - 1], "columns ascend");
    riga::Plan twice;
    check(twice.build_realform(r) != 0, "no real form of a real form");
  }
}

void dense_eig(std::mt19937_64& rng) {
  std::normal_distribution<double> g;
  for (int n : {1, 2, 7, 33, 80}) {
    std::vector<double> A((size_t)n * n), T, Q;
    for (auto& x : A) x = g(rng);
    check(riga::schur_real(n, A.data(), T, Q) == 0, "real Schur form");
    double err = 0.0, an = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k)
          for (int l = 0; l < n; ++l) s += Q[i + (size_t)k * n] * T[k + (size_t)l * n] * Q[j + (size_t)l * n];
        err = std::max(err, std::abs(s - A[i + (size_t)j * n]));
        an = std::max(an, std::abs(A[i + (size_t)j * n]));
      }
    check(err <= 1e-12 * an * n, "Q T Q^T reproduces A");
    std::vector<char> keep(n, 0);
    for (int i = 0; i < n; i += 3) keep[i] = 1;
    // keep whole 2x2 blocks
    for (int i = 0; i + 1 < n; ++i)
      if (T[(i + 1) + (size_t)i * n] != 0.0 && (keep[i] || keep[i + 1])) keep[i] = keep[i + 1] = 1;
    std::vector<double> T2 = T, Q2 = Q;
    const int r = riga::schur_select_real(n, T2, Q2, keep);
    check(r != 0, "reordering returns a kept dimension or -1");
    std::vector<riga::cplx> th, Y;
    riga::schur_real_eigvals(n, T, th);
    riga::schur_eigvecs_real(n, T, Q, th, Y, 1e-10);
    check((int)Y.size() == n * n, "eigenvectors formed");
  }
}

void krylov_schur_cycle(std::mt19937_64& rng) {
  std::normal_distribution<double> g;
  const int b = 2, m = 40, nev = 10, ldh = m + 2 * b, k = m;
  std::vector<double> H((size_t)ldh * ldh, 0.0);
  // block upper Hessenberg H_k with a residual block below it
  for (int c = 0; c < k; ++c)
    for (int r = 0; r <= std::min(k + b - 1, c + b); ++r) H[r + (size_t)c * ldh] = g(rng) / (1.0 + 0.1 * r);
  riga::KsCycle cyc;
  check(riga::ks_ritz(H, ldh, k, b, nev, 1e-12, cyc) == 0, "Rayleigh-Ritz");
  check(cyc.nw >= nev, "wanted values cover nev");
  riga::ks_restart(H, ldh, k, b, m, nev, 0, cyc);
  check(cyc.r >= nev && cyc.r + b <= m, "kept dimension");
  check((int)cyc.Qe.size() == (k + b) * (cyc.r + b), "restart combination size");
  check(riga::ks_ritz(cyc.Hn, ldh, cyc.r, b, nev, 1e-12, cyc) == 0, "Rayleigh-Ritz after the restart");
  riga::ks_ritz_vectors(cyc);
}

void pool() {
  riga::HostPool& P = riga::HostPool::get();
  for (int rep = 0; rep < 20; ++rep) {
    std::vector<int> hit(1000, 0);
    std::atomic<long> sum{0};
    P.run(1000, [&](int i) {
      hit[i] += 1;
      sum += i;
    });
    bool once = true;
    for (int h : hit) once &= h == 1;
    check(once && sum.load() == 999L * 1000 / 2, "every index once");
  }
  bool caught = false;
  try {
    P.run(200, [&](int i) {
      if (i == 17) throw std::runtime_error("job 17");
    });
  } catch (const std::runtime_error& e) {
    caught = std::strcmp(e.what(), "job 17") == 0;
  }
  check(caught, "a throwing job is rethrown on the caller");
  std::atomic<int> cnt{0};
  P.run(64, [&](int) { ++cnt; });
  check(cnt.load() == 64, "the pool runs again after an exception");
}
// The symmetric eigensolver of the Lanczos slices: A = Q diag(d) Q^T with a
// known spectrum spread over eight decades, both signs and a double value
// (Q a product of random Householder reflectors); the computed values must
// match d sorted and the vectors must be orthonormal with small residuals.
void symmetric_eig(std::mt19937_64& rng) {
  std::normal_distribution<double> g;
  for (int n : {1, 2, 9, 40, 84, 160}) {
    std::vector<double> d(n), Q((size_t)n * n, 0.0), A((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = (i % 2 ? -1.0 : 1.0) * std::pow(10.0, -4.0 + 8.0 * i / std::max(1, n - 1));
    if (n > 3) d[3] = d[2];
    for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
    for (int r = 0; r < 3; ++r) {
      std::vector<double> v(n);
      double vv = 0.0;
      for (auto& x : v) { x = g(rng); vv += x * x; }
      for (int i = 0; i < n; ++i) {   // Q <- Q (I - 2 v v^T / v^T v)
        double qv = 0.0;
        for (int k = 0; k < n; ++k) qv += Q[i + (size_t)k * n] * v[k];
        for (int k = 0; k < n; ++k) Q[i + (size_t)k * n] -= 2.0 * qv * v[k] / vv;
      }
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += Q[i + (size_t)k * n] * d[k] * Q[j + (size_t)k * n];
        A[i + (size_t)j * n] = s;
      }
    std::vector<double> w, Z;
    check(riga::sym_eig_jacobi(n, A.data(), w, Z) >= 0, "Jacobi converges");
    std::vector<double> ds = d;
    std::sort(ds.begin(), ds.end());
    double ev = 0.0, orth = 0.0, res = 0.0;
    for (int i = 0; i < n; ++i) ev = std::max(ev, std::abs(w[i] - ds[i]));
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0, r = 0.0;
        for (int k = 0; k < n; ++k) s += Z[k + (size_t)a * n] * Z[k + (size_t)b * n];
        orth = std::max(orth, std::abs(s - (a == b ? 1.0 : 0.0)));
        for (int k = 0; k < n; ++k) r += A[a + (size_t)k * n] * Z[k + (size_t)b * n];
        res = std::max(res, std::abs(r - w[b] * Z[a + (size_t)b * n]));
      }
    // A itself carries the rounding of Q diag(d) Q^T, about n eps max|d|
    const double scale = 1e-4 * std::pow(10.0, 8.0);
    check(ev <= 1e-14 * n * scale, "Jacobi eigenvalues");
    check(orth <= 1e-13 * n, "Jacobi vectors orthonormal");
    check(res <= 1e-14 * n * scale, "Jacobi residuals");
  }
}

}  // namespace

int main(int argc, char** argv) {
  const bool tsan = argc > 1 && std::strcmp(argv[1], "tsan") == 0;
  std::mt19937_64 rng(12345);
  if (!tsan) {
    plans();
    realform_plans();
    dense_eig(rng);
    symmetric_eig(rng);
    krylov_schur_cycle(rng);
  }
  pool();
  if (failures) return 1;
  std::printf("host checks ok (%s)\n", tsan ? "tsan" : "asan+ubsan");
  return 0;
}
