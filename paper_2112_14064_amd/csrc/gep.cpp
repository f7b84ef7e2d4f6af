// The undamped case C = 0: the QEP of eq. QuadEig reduces to the Hermitian
// definite pencil K u = mu M u (lam^2 = -mu), whose eigenvalues are real, so
// the spectrum can be sliced (Sec. 4.1.4).  Per slice:
//   - the signed factorization K - s M = L S L^T (S = diag(+-1)) of the
//     multifrontal tree, whose negative pivots count the eigenvalues below s
//     (Sylvester's law of inertia);
//   - thick-restart block Lanczos on the shift-and-invert operator
//     (K - s M)^{-1} M with M-orthonormal bases (the Lanczos remark of Sec.
//     4.1.2: the projected matrix of this operator is symmetric), with full
//     reorthogonalisation (classical Gram--Schmidt applied twice) and
//     Krylov--Schur restarts, which for a symmetric projected matrix keep a
//     diagonal block plus one coupling block row (Sec. 4.1.3).
// Every N-sized operation runs in the device kernels (sweeps, sum-factorised
// mass products, multi-dots, updates, tall products); the host holds the
// projected matrix (at most 256 x 256) and the slice bookkeeping.
#include "problem.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

using namespace riga::detail;

namespace {

struct Lanczos {
  riga_problem* h;
  int64_t N;
  int m, b, ldh;
  double tol;
  std::vector<double> H;   // ldh x ldh, column-major
  int64_t n_op = 0, n_restart = 0;

  double& Hat(int r, int c) { return H[r + (size_t)c * ldh]; }

  void to_host(const double* d, std::vector<double>& out, size_t n) {
    out.resize(n);
    ck(hipMemcpyAsync(out.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
  }

  // Out (N x kout) = In (N x kin) Q (kin x kout, host, column-major).
  void tall(const double* in, int kin, const std::vector<double>& Q, int kout, double* out) {
    double* dQ = h->d_small + (size_t)3 * ldh * b;
    ck(hipMemcpyAsync(dQ, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    riga::launch_gemm_tall(N, in, N, kin, dQ, kout, out, N, h->st);
    ck(hipStreamSynchronize(h->st));   // dQ is staged again by the next call
  }

  // M-orthonormalise the block (R, MR = M R) against V[:, 0:nc] (CGS twice),
  // store it as V[:, nc:nc+b], W[:, nc:nc+b]; hsum (nc x b) the projection
  // coefficients, Rb (b x b, upper) with block = V[:, 0:nc] hsum + V[:, nc:nc+b] Rb.
  // Returns false when the block lost rank (an invariant subspace).
  bool orthonormalize(int nc, std::vector<double>& hsum, std::vector<double>& Rb) {
    double* dh = h->d_small;
    double* dG = h->d_small + (size_t)2 * ldh * b;
    double* R = h->Ru;
    double* MR = h->MRl;
    hsum.assign((size_t)nc * b, 0.0);
    if (nc > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        double* hp = dh + (size_t)pass * ldh * b;
        riga::launch_dots(N, nc, h->Wl, nullptr, N, b, R, nullptr, N, h->d_part, hp, h->st);
        riga::launch_cgs_update(N, nc, b, hp, h->Vu, R, h->Wl, MR, nullptr, nullptr, N, N, nullptr, h->st);
      }
      std::vector<double> hh;
      to_host(dh, hh, (size_t)2 * ldh * b);
      for (int c = 0; c < nc; ++c)
        for (int q = 0; q < b; ++q)
          hsum[c + (size_t)q * nc] = hh[(size_t)c * b + q] + hh[(size_t)ldh * b + (size_t)c * b + q];
    }
    riga::launch_dots(N, b, R, nullptr, N, b, MR, nullptr, N, h->d_part, dG, h->st);
    std::vector<double> G;
    to_host(dG, G, (size_t)b * b);
    for (int c = 0; c < b; ++c)
      for (int q = c + 1; q < b; ++q) {
        const double v = 0.5 * (G[c * b + q] + G[q * b + c]);
        G[c * b + q] = G[q * b + c] = v;
      }
    // squared M-norms of the columns before the projection, for the rank test
    std::vector<double> n0(b);
    for (int q = 0; q < b; ++q) {
      double s = G[q * b + q];
      for (int c = 0; c < nc; ++c) s += hsum[c + (size_t)q * nc] * hsum[c + (size_t)q * nc];
      n0[q] = s;
    }
    Rb.assign((size_t)b * b, 0.0);
    for (int j = 0; j < b; ++j)
      for (int i = 0; i <= j; ++i) {
        double s = G[i + (size_t)j * b];
        for (int k = 0; k < i; ++k) s -= Rb[k + (size_t)i * b] * Rb[k + (size_t)j * b];
        if (i == j) {
          if (!(s > 1e-24 * n0[j])) return false;
          Rb[j + (size_t)j * b] = std::sqrt(s);
        } else {
          Rb[i + (size_t)j * b] = s / Rb[i + (size_t)i * b];
        }
      }
    const std::vector<double> Ri = upper_inverse(b, Rb);
    tall(R, b, Ri, b, h->Vu + (size_t)nc * N);
    tall(MR, b, Ri, b, h->Wl + (size_t)nc * N);
    return true;
  }

  // R = (K - s M)^{-1} W[:, k:k+b] = S V[:, k:k+b]; MR = M R.
  void apply(int k) {
    solve_levels(h, b, h->Wl + (size_t)k * N, N, h->Ru, N, nullptr, nullptr, 0, 0.0);
    mass_product(h, b, h->Ru, h->MRl);
    n_op += b;
  }

  // Start block: the library's counter-based generator, M-orthonormalised.
  bool start(uint64_t seed) {
    riga::launch_random_fill(h->Ru, N, b, N, seed, h->st);
    mass_product(h, b, h->Ru, h->MRl);
    std::vector<double> hs, Rb;
    return orthonormalize(0, hs, Rb);
  }

  // Extend the basis from k kept columns to m: block steps of eq. Arnoldi.
  // Returns false on a breakdown.
  bool expand(int k) {
    std::vector<double> hs, Rb;
    for (; k + b <= m; k += b) {
      apply(k);
      const int nc = k + b;
      if (!orthonormalize(nc, hs, Rb)) return false;
      for (int c = 0; c < nc; ++c)
        for (int q = 0; q < b; ++q) Hat(c, k + q) = hs[c + (size_t)q * nc];
      for (int i = 0; i < b; ++i)
        for (int q = 0; q < b; ++q) Hat(nc + i, k + q) = Rb[i + (size_t)q * b];
    }
    return true;
  }
};

// Eigenpairs of the slice [lo, hi) that holds `cnt` eigenvalues: the Lanczos
// run at the shift s (factored) for the `want` values of theta of largest
// modulus, those with mu = s + 1/theta in [lo, hi) kept (at most `room`).
// Returns the pairs found (mu ascending); their Ritz vectors go to U (device,
// ndof x found) when not null.  A Ritz pair counts as converged when its
// residual estimate is below tol times the largest |theta| (the norm of the
// operator, which bounds the rounding of the computed Krylov relation): a
// shift close to one eigenvalue makes that |theta| large, and a bound
// relative to each |theta| could then not be met for the others.
int solve_slice(riga_problem* h, double s, double lo, double hi, int want, int room, const riga_options& o,
                double* mu_out, double* U, int64_t* n_op, int64_t* n_restart, bool* ok) {
  const int64_t N = h->N();
  Lanczos L;
  L.h = h;
  L.N = N;
  L.b = o.block > 0 ? o.block : 2;
  want = (int)std::min<int64_t>(want, std::min<int64_t>(N - L.b, 256 - 4 * L.b) / 2);
  int m = std::max(2 * want, want + 2 * L.b);
  m = std::max(m, 20);
  m = (m + L.b - 1) / L.b * L.b;
  m = std::min<int>(m, (int)std::min<int64_t>(256 - 2 * L.b, N - L.b) / L.b * L.b);
  L.m = m;
  L.ldh = m + 2 * L.b;
  L.tol = o.tol > 0 ? o.tol : 1e-12;
  const int maxit = o.maxit > 0 ? o.maxit : 200;
  ensure_krylov(h, L.ldh, L.b);
  L.H.assign((size_t)L.ldh * L.ldh, 0.0);
  *ok = false;
  if (!L.start(o.seed + (uint64_t)std::llround(std::abs(s) * 1e6))) return 0;
  int k = 0;
  std::vector<double> theta, Y;
  std::vector<int> order;
  for (int it = 0; it <= maxit; ++it) {
    if (!L.expand(k)) return 0;
    // Rayleigh--Ritz on the symmetric projected matrix H[0:m, 0:m]
    std::vector<double> Hm((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) Hm[i + (size_t)j * m] = 0.5 * (L.Hat(i, j) + L.Hat(j, i));
    if (riga::sym_eig_jacobi(m, Hm.data(), theta, Y) < 0) return 0;
    order.resize(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return std::abs(theta[a]) > std::abs(theta[c]); });
    // On a curl-conforming space the gradients form the eigenvalue mu = 0 of
    // huge multiplicity (theta = -1/s).  No slice contains it, yet from a
    // shift s below the next eigenvalue's distance its |theta| ranks among
    // the values asked for beyond the slice's own; its Ritz values, which
    // rounding keeps replenishing, go last: they are neither waited for nor
    // kept at a restart (the cluster rule would keep them all and leave one
    // block step per restart).
    if (h->plan.kind != riga::SPACE_H1)
      std::stable_partition(order.begin(), order.end(),
                            [&](int j) { return std::abs(s + 1.0 / theta[j]) > 1e-6 * std::abs(s); });
    // residual estimates ||E y|| with E = H[m:m+b, m-b:m]
    auto resid = [&](int j) {
      double r2 = 0.0;
      for (int i = 0; i < L.b; ++i) {
        double s2 = 0.0;
        for (int q = 0; q < L.b; ++q) s2 += L.Hat(m + i, m - L.b + q) * Y[(m - L.b + q) + (size_t)j * m];
        r2 += s2 * s2;
      }
      return std::sqrt(r2);
    };
    int conv = 0;
    const double tmax = std::abs(theta[order[0]]);
    while (conv < want && resid(order[conv]) <= L.tol * tmax) ++conv;
    if (conv >= want || it == maxit) {
      // Ritz values in the slice
      std::vector<int> sel;
      for (int i = 0; i < (conv >= want ? want : conv); ++i) {
        const double muv = s + 1.0 / theta[order[i]];
        if (muv >= lo && muv < hi && (int)sel.size() < room) sel.push_back(order[i]);
      }
      std::sort(sel.begin(), sel.end(), [&](int a, int c) { return s + 1.0 / theta[a] < s + 1.0 / theta[c]; });
      const int nf = (int)sel.size();
      for (int i = 0; i < nf; ++i) mu_out[i] = s + 1.0 / theta[sel[i]];
      if (U != nullptr && nf > 0) {
        std::vector<double> Q((size_t)m * nf);
        for (int i = 0; i < nf; ++i)
          for (int r = 0; r < m; ++r) Q[r + (size_t)i * m] = Y[r + (size_t)sel[i] * m];
        L.tall(h->Vu, m, Q, nf, U);
      }
      *n_op += L.n_op;
      *n_restart += L.n_restart;
      *ok = conv >= want;
      return nf;
    }
    // restart: keep the p Ritz vectors of largest |theta| (whole clusters)
    int p = std::min(m - L.b, want + (m - want) / 2);
    p = std::max(p, std::min(m - L.b, conv + 1));
    while (p < m - L.b &&
           std::abs(std::abs(theta[order[p]]) - std::abs(theta[order[p - 1]])) <= 1e-9 * std::abs(theta[order[p - 1]]))
      ++p;
    // whole blocks: the block steps after the restart must end exactly at m
    p = std::min(m - L.b, (p + L.b - 1) / L.b * L.b);
    std::vector<double> Q((size_t)m * p);
    for (int i = 0; i < p; ++i)
      for (int r = 0; r < m; ++r) Q[r + (size_t)i * m] = Y[r + (size_t)order[i] * m];
    L.tall(h->Vu, m, Q, p, h->Vu2);
    L.tall(h->Wl, m, Q, p, h->Wl2);
    ck(hipMemcpyAsync(h->Vu2 + (size_t)p * N, h->Vu + (size_t)m * N, (size_t)L.b * N * sizeof(double),
                      hipMemcpyDeviceToDevice, h->st));
    ck(hipMemcpyAsync(h->Wl2 + (size_t)p * N, h->Wl + (size_t)m * N, (size_t)L.b * N * sizeof(double),
                      hipMemcpyDeviceToDevice, h->st));
    std::swap(h->Vu, h->Vu2);
    std::swap(h->Wl, h->Wl2);
    std::vector<double> Hn((size_t)L.ldh * L.ldh, 0.0);
    for (int i = 0; i < p; ++i) {
      Hn[i + (size_t)i * L.ldh] = theta[order[i]];
      for (int r = 0; r < L.b; ++r) {
        double s2 = 0.0;
        for (int q = 0; q < L.b; ++q) s2 += L.Hat(m + r, m - L.b + q) * Y[(m - L.b + q) + (size_t)order[i] * m];
        Hn[(p + r) + (size_t)i * L.ldh] = s2;
      }
    }
    L.H.swap(Hn);
    k = p;
    ++L.n_restart;
  }
  return 0;
}

// mu[j] = u_j^T K u_j / u_j^T M u_j for the n columns of U.  A Ritz value
// s + 1/theta far from its slice's shift carries the rounding of the shifted
// solves amplified by (mu - s)^2 |theta_max|; the Rayleigh quotient's error is
// quadratic in the eigenvector's.  Two columns per pass: K u and M u side by
// side in d_tmp2 (N x 4), the four products of each column with them in one
// reduction; one synchronisation per group that d_small holds.
void rayleigh_quotients(riga_problem* h, int n, const double* U, double* mu) {
  const int64_t N = h->N();
  double* T = h->d_tmp2;
  const int per_group = std::max(1, (int)((4 * h->kw_cols * h->kw_cols + 64) / 8));
  for (int g0 = 0; g0 < n; g0 += 2 * per_group) {
    const int g1 = std::min(n, g0 + 2 * per_group);
    for (int j = g0; j < g1; j += 2) {
      const int c = std::min(2, g1 - j);
      const double* u = U + (size_t)j * N;
      // K u_c at T + 2cN, M u_c at T + (2c + 1)N
      riga::launch_spmv(h->ds, N, c, h->d_K, 1.0, u, N, T, 2 * N, nullptr, 0, 0.0, nullptr, 0, h->st);
      riga::launch_spmv(h->ds, N, c, h->d_M, 1.0, u, N, T + N, 2 * N, nullptr, 0, 0.0, nullptr, 0, h->st);
      riga::launch_dots(N, c, u, nullptr, N, 2 * c, T, nullptr, N, h->d_part, h->d_small + 4 * (j - g0), h->st);
    }
    std::vector<double> out((size_t)4 * (g1 - g0 + 1));
    ck(hipMemcpyAsync(out.data(), h->d_small, (size_t)4 * (g1 - g0) * sizeof(double), hipMemcpyDeviceToHost, h->st));
    ck(hipStreamSynchronize(h->st));
    for (int jc = g0; jc < g1; jc += 2) {
      const int cc = std::min(2, g1 - jc), nq = 2 * cc;
      const double* o = out.data() + 4 * (jc - g0);   // o[c nq + q]: column c times T column q
      for (int c = 0; c < cc; ++c) {
        const double uku = o[c * nq + 2 * c], umu = o[c * nq + 2 * c + 1];
        if (umu > 0.0 && std::isfinite(uku)) mu[jc + c] = uku / umu;
      }
    }
  }
}

// Near-degenerate groups of returned values (consecutive, spacing below
// 1e-6 relative, at most 8): a slice resolves its Ritz vectors to its own
// tolerance relative to its largest |theta|, and vectors of values closer than
// that can be mixtures within their group, whose span is nevertheless accurate.
// Rayleigh-Ritz with K and M on each group's span (a k x k definite pencil,
// Cholesky of the M block and cyclic Jacobi) separates them: the values and
// vectors of the group are replaced by its Ritz pairs (M-orthonormal).  A
// group whose values already agree to 1e-12 is left alone (an exact multiple
// eigenvalue: any basis of its space is exact).  All groups in one pass: the
// products [K U_g | M U_g] side by side, their Gram blocks in one download,
// the rotations in one upload.
void group_rayleigh_ritz(riga_problem* h, int n, double* U, double* mu) {
  const int64_t N = h->N();
  std::vector<std::pair<int, int>> groups;   // (first column, size)
  int cols = 0;
  for (int i = 0; i < n;) {
    int j = i + 1;
    while (j < n && j - i < 8 && mu[j] - mu[j - 1] <= 1e-6 * std::abs(mu[j])) ++j;
    if (j - i >= 2 && mu[j - 1] - mu[i] > 1e-12 * std::abs(mu[j - 1])) {
      groups.push_back({i, j - i});
      cols += j - i;
    }
    i = j;
  }
  if (groups.empty()) return;
  if (h->grp_cols < cols) {
    if (h->d_grp) h->dfree(h->d_grp);
    if (h->d_grpG) h->dfree(h->d_grpG);
    h->d_grp = h->dalloc<double>((size_t)2 * cols * N);
    h->d_grpG = h->dalloc<double>((size_t)16 * cols + 64);
    h->grp_cols = cols;
  }
  // products and Gram blocks: group g at column offset 2 o_g of d_grp and at
  // 2 o_g k_g of d_grpG
  std::vector<int> off(groups.size());
  int o = 0, go = 0;
  std::vector<int> goff(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    const int i = groups[g].first, k = groups[g].second;
    off[g] = o;
    goff[g] = go;
    double* Uc = U + (size_t)i * N;
    double* KM = h->d_grp + (size_t)2 * o * N;
    riga::launch_spmv(h->ds, N, k, h->d_K, 1.0, Uc, N, KM, N, nullptr, 0, 0.0, nullptr, 0, h->st);
    riga::launch_spmv(h->ds, N, k, h->d_M, 1.0, Uc, N, KM + (size_t)k * N, N, nullptr, 0, 0.0, nullptr, 0, h->st);
    for (int q0 = 0; q0 < 2 * k; q0 += 4) {
      const int nq = std::min(4, 2 * k - q0);
      riga::launch_dots(N, k, Uc, nullptr, N, nq, KM + (size_t)q0 * N, nullptr, N, h->d_part,
                        h->d_grpG + go + (size_t)k * q0, h->st);
    }
    o += k;
    go += 2 * k * k;
  }
  std::vector<double> G((size_t)go);
  ck(hipMemcpyAsync(G.data(), h->d_grpG, G.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
  ck(hipStreamSynchronize(h->st));
  std::vector<double> Yall((size_t)go / 2, 0.0);   // k x k per group, at goff / 2
  std::vector<char> done(groups.size(), 0);
  for (size_t g = 0; g < groups.size(); ++g) {
    const int i = groups[g].first, k = groups[g].second;
    const double* Gg = G.data() + goff[g];
    // chunk q0 holds out[c nq + q] for column c of U_g and column q0 + q
    std::vector<double> Kc((size_t)k * k), Mc((size_t)k * k);
    for (int q0 = 0; q0 < 2 * k; q0 += 4) {
      const int nq = std::min(4, 2 * k - q0);
      for (int c = 0; c < k; ++c)
        for (int q = 0; q < nq; ++q) {
          const int col = q0 + q;
          const double v = Gg[(size_t)k * q0 + (size_t)c * nq + q];
          if (col < k) Kc[c + (size_t)col * k] = v; else Mc[c + (size_t)(col - k) * k] = v;
        }
    }
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < a; ++b) {
        const double ks = 0.5 * (Kc[a + (size_t)b * k] + Kc[b + (size_t)a * k]);
        const double ms = 0.5 * (Mc[a + (size_t)b * k] + Mc[b + (size_t)a * k]);
        Kc[a + (size_t)b * k] = Kc[b + (size_t)a * k] = ks;
        Mc[a + (size_t)b * k] = Mc[b + (size_t)a * k] = ms;
      }
    // Mc = L L^T; the pencil becomes L^{-1} Kc L^{-T}
    std::vector<double> L((size_t)k * k, 0.0);
    bool spd = true;
    for (int c = 0; c < k && spd; ++c) {
      double d = Mc[c + (size_t)c * k];
      for (int q = 0; q < c; ++q) d -= L[c + (size_t)q * k] * L[c + (size_t)q * k];
      if (!(d > 0.0)) { spd = false; break; }
      d = std::sqrt(d);
      L[c + (size_t)c * k] = d;
      for (int r = c + 1; r < k; ++r) {
        double v = Mc[r + (size_t)c * k];
        for (int q = 0; q < c; ++q) v -= L[r + (size_t)q * k] * L[c + (size_t)q * k];
        L[r + (size_t)c * k] = v / d;
      }
    }
    if (!spd) continue;
    auto lsolve = [&](std::vector<double>& X) {   // X <- L^{-1} X (k columns)
      for (int col = 0; col < k; ++col)
        for (int r = 0; r < k; ++r) {
          double v = X[r + (size_t)col * k];
          for (int q = 0; q < r; ++q) v -= L[r + (size_t)q * k] * X[q + (size_t)col * k];
          X[r + (size_t)col * k] = v / L[r + (size_t)r * k];
        }
    };
    std::vector<double> A = Kc;
    lsolve(A);
    std::vector<double> At((size_t)k * k);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) At[a + (size_t)b * k] = A[b + (size_t)a * k];
    lsolve(At);
    std::vector<double> w, Z;
    if (riga::sym_eig_jacobi(k, At.data(), w, Z) < 0) continue;
    std::vector<int> ord(k);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] < w[b]; });
    double* Y = Yall.data() + goff[g] / 2;   // L^{-T} Z, columns in ascending order of w
    for (int c = 0; c < k; ++c) {
      const int oc = ord[c];
      for (int r = k - 1; r >= 0; --r) {
        double v = Z[r + (size_t)oc * k];
        for (int q = r + 1; q < k; ++q) v -= L[q + (size_t)r * k] * Y[q + (size_t)c * k];
        Y[r + (size_t)c * k] = v / L[r + (size_t)r * k];
      }
      mu[i + c] = w[oc];
    }
    done[g] = 1;
  }
  // rotations: U_g <- U_g Y_g through the group's first k product columns
  ck(hipMemcpyAsync(h->d_grpG, Yall.data(), Yall.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
  for (size_t g = 0; g < groups.size(); ++g) {
    if (!done[g]) continue;
    const int i = groups[g].first, k = groups[g].second;
    double* Uc = U + (size_t)i * N;
    double* Wg = h->d_grp + (size_t)2 * off[g] * N;
    riga::launch_gemm_tall(N, Uc, N, k, h->d_grpG + goff[g] / 2, k, Wg, N, h->st);
    ck(hipMemcpyAsync(Uc, Wg, (size_t)k * N * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  }
  ck(hipStreamSynchronize(h->st));   // Yall is host memory read by the upload
}

// Ascending order of the n values, the columns of U permuted with them (a
// polished value can pass a neighbour it was within rounding of).
void order_pairs(riga_problem* h, int n, double* U, double* mu) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return mu[a] < mu[c]; });
  const int64_t N = h->N();
  const size_t bytes = (size_t)N * sizeof(double);
  std::vector<double> sorted(n);
  std::vector<char> seen(n, 0);
  for (int i = 0; i < n; ++i) sorted[i] = mu[perm[i]];
  // column i of the result is column perm[i]: follow each cycle once through
  // one spare column
  for (int i = 0; i < n; ++i) {
    if (seen[i] || perm[i] == i) { seen[i] = 1; continue; }
    ck(hipMemcpyAsync(h->d_tmp, U + (size_t)i * N, bytes, hipMemcpyDeviceToDevice, h->st));
    int j = i;
    while (perm[j] != i) {
      ck(hipMemcpyAsync(U + (size_t)j * N, U + (size_t)perm[j] * N, bytes, hipMemcpyDeviceToDevice, h->st));
      seen[j] = 1;
      j = perm[j];
    }
    ck(hipMemcpyAsync(U + (size_t)j * N, h->d_tmp, bytes, hipMemcpyDeviceToDevice, h->st));
    seen[j] = 1;
  }
  for (int i = 0; i < n; ++i) mu[i] = sorted[i];
}

}  // namespace

extern "C" {

riga_status riga_factor_gep(riga_problem* h, double shift, int64_t* neg_count, int64_t* bad_pivot) {
  if (bad_pivot) *bad_pivot = -1;
  if (!h || !std::isfinite(shift)) return RIGA_ERR_INVALID_ARG;
  if (!h->assembled) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    int64_t negs = 0;
    const riga_status rc = factor_gep_all(h, shift, bad_pivot, &negs);
    if (neg_count) *neg_count = negs;
    return rc;
  });
}

riga_status riga_gep_slice(riga_problem* h, double a, double b, int max_slice, const riga_options* opt, int cap,
                           double* mu, double* U, double* resid, int64_t* count, int* found, int64_t* stats) {
  if (count) *count = 0;
  if (found) *found = 0;
  if (!h || !opt || !mu || !count || !found || cap < 0 || !(a < b) || !std::isfinite(a) || !std::isfinite(b))
    return RIGA_ERR_INVALID_ARG;
  if (max_slice == 0) max_slice = 40;
  if (max_slice < 2 || opt->block < 0 || opt->block > 4 || opt->v0 != nullptr) return RIGA_ERR_INVALID_ARG;
  if (h->plan.kind != riga::SPACE_H1 && !(a > 0.0)) return RIGA_ERR_INVALID_ARG;   // the null space
  if (!h->assembled) return RIGA_ERR_STATE;
  return run([&]() -> riga_status {
    ck(hipSetDevice(h->device));
    const auto t0 = std::chrono::steady_clock::now();
    int64_t nfac = 0, n_op = 0, n_restart = 0;
    double t_fac = 0.0;
    // nu(s) at a shift, moving it by a relative 1e-9 when it falls on an
    // eigenvalue to working precision (a zero pivot)
    auto inertia = [&](double& s, int64_t* nu) -> riga_status {
      for (int attempt = 0; attempt < 4; ++attempt) {
        int64_t bad = -1;
        const riga_status rc = factor_gep_all(h, s, &bad, nu);
        ++nfac;
        t_fac += h->stats.t_factor_ms;
        if (rc == RIGA_OK) return RIGA_OK;
        if (rc != RIGA_ERR_NOT_SPD) return rc;
        s += 1e-9 * std::max(std::abs(s), 1.0) * (attempt + 1);
      }
      return RIGA_ERR_NOT_SPD;
    };
    struct Slice { double lo, hi; int64_t nlo, nhi; };
    double lo = a, hi = b;
    int64_t nlo = 0, nhi = 0;
    riga_status rc = inertia(lo, &nlo);
    if (rc != RIGA_OK) return rc;
    rc = inertia(hi, &nhi);
    if (rc != RIGA_OK) return rc;
    *count = nhi - nlo;
    if (*count > cap) return RIGA_ERR_INVALID_ARG;
    // bisect until every slice holds at most max_slice eigenvalues.  A vector
    // space's pencil has the gradients as a null space of huge multiplicity:
    // seen from the midpoint s of a slice [l, r) they are the value
    // theta = -1/s, against |theta| >= 2/(r - l) for the slice's own values.
    // The slice solver sets converged null Ritz values aside, but Ritz values
    // that still mix the null space with the slice's vectors would compete
    // with its smallest |theta|; its slices are therefore also halved until
    // r - l <= l / 2 (the null cluster then stays below a fifth of every
    // wanted |theta|)
    const double rho = h->plan.kind != riga::SPACE_H1 ? 0.5 : 0.0;
    std::vector<Slice> todo{{lo, hi, nlo, nhi}}, done;
    while (!todo.empty()) {
      Slice sl = todo.back();
      todo.pop_back();
      const bool narrow = rho == 0.0 || (sl.lo > 0.0 && sl.hi - sl.lo <= rho * sl.lo);
      // a slice narrower than 1e-10 relative (a cluster of more than max_slice
      // equal eigenvalues) is solved as it is
      if (sl.nhi == sl.nlo || (sl.nhi - sl.nlo <= max_slice && narrow) ||
          sl.hi - sl.lo <= 1e-10 * std::max(std::abs(sl.hi), 1e-300)) {
        if (sl.nhi > sl.nlo) done.push_back(sl);
        continue;
      }
      double mid = 0.5 * (sl.lo + sl.hi);
      int64_t nm = 0;
      rc = inertia(mid, &nm);
      if (rc != RIGA_OK) return rc;
      if (nm < sl.nlo || nm > sl.nhi) return RIGA_ERR_NOT_SPD;   // counts must be monotone
      todo.push_back({mid, sl.hi, nm, sl.nhi});
      todo.push_back({sl.lo, mid, sl.nlo, nm});
    }
    std::sort(done.begin(), done.end(), [](const Slice& x, const Slice& y) { return x.lo < y.lo; });
    int nout = 0;
    bool all_ok = true;
    riga_options o = *opt;
    for (const Slice& sl : done) {
      const int cnt = (int)(sl.nhi - sl.nlo);
      // the midpoint first: the slice's cnt eigenvalues are then the cnt
      // nearest to it; should the slice come out incomplete (a run that did
      // not converge), again from shifts off the middle, asking for more values
      int nf = 0;
      for (int attempt = 0; attempt < 3; ++attempt) {
        const double frac = attempt == 0 ? 0.5 : (attempt == 1 ? 0.35 : 0.65);
        double s = sl.lo + frac * (sl.hi - sl.lo);
        int64_t ns = 0;
        rc = inertia(s, &ns);
        if (rc != RIGA_OK) return rc;
        bool ok = false;
        nf = solve_slice(h, s, sl.lo, sl.hi, cnt + 2 + attempt * cnt, cap - nout, o, mu + nout,
                         U ? U + (size_t)nout * h->N() : nullptr, &n_op, &n_restart, &ok);
        // the slice is complete when its converged values number its inertia count
        if (nf == cnt) break;
      }
      if (nf != cnt) all_ok = false;
      nout += nf;
    }
    *found = nout;
    if (U != nullptr && nout > 0) {
      rayleigh_quotients(h, nout, U, mu);
      order_pairs(h, nout, U, mu);
      group_rayleigh_ritz(h, nout, U, mu);
    }
    if (resid != nullptr && U != nullptr && nout > 0) {
      ensure_norms(h);
      const double nk = h->norms[0], nm = h->norms[2];
      const int64_t N = h->N();
      double* T = h->d_tmp2;
      double* out = h->d_small;
      for (int j = 0; j < nout; ++j) {
        const double* u = U + (size_t)j * N;
        riga::launch_spmv(h->ds, N, 1, h->d_M, -mu[j], u, N, T, N, nullptr, 0, 0.0, nullptr, 0, h->st);
        riga::launch_spmv(h->ds, N, 1, h->d_K, 1.0, u, N, T, N, T, N, 1.0, nullptr, 0, h->st);
        riga::launch_dots(N, 1, T, nullptr, N, 1, T, nullptr, N, h->d_part, out + 2 * j, h->st);
        riga::launch_dots(N, 1, u, nullptr, N, 1, u, nullptr, N, h->d_part, out + 2 * j + 1, h->st);
      }
      std::vector<double> rr((size_t)2 * nout);
      ck(hipMemcpyAsync(rr.data(), out, rr.size() * sizeof(double), hipMemcpyDeviceToHost, h->st));
      ck(hipStreamSynchronize(h->st));
      for (int j = 0; j < nout; ++j)
        resid[j] = std::sqrt(rr[2 * j]) / ((nk + std::abs(mu[j]) * nm) * std::sqrt(rr[2 * j + 1]));
    }
    ck(hipStreamSynchronize(h->st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    h->stats.t_factor_ms = t_fac;
    h->stats.t_eigs_ms = ms - t_fac;
    h->stats.n_fb = n_op;
    h->stats.n_it = n_restart;
    if (stats) {
      stats[0] = nfac;
      stats[1] = (int64_t)done.size();
      stats[2] = n_op;
      stats[3] = n_restart;
    }
    return (all_ok && nout == *count) ? RIGA_OK : RIGA_WARN_NOT_CONVERGED;
  });
}

}  // extern "C"
