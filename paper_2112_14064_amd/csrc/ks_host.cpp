#include "ks_host.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace riga {

int ks_ritz(const std::vector<double>& H, int ldh, int k, int b, int nev, double tol, KsCycle& c) {
  auto Hat = [&](int r, int col) { return H[r + (size_t)col * ldh]; };
  std::vector<double> Hk((size_t)k * k);
  for (int col = 0; col < k; ++col)
    for (int r = 0; r < k; ++r) Hk[r + (size_t)col * k] = Hat(r, col);
  if (schur_real(k, Hk.data(), c.TR, c.QR) != 0) return -1;
  c.T.clear();   // the complex Schur form is formed only if a restart needs it
  c.Z.clear();
  schur_real_eigvals(k, c.TR, c.theta);
  // sort by |theta| descending (= |lam - sigma| ascending), clusters kept together
  c.ord.resize(k);
  std::iota(c.ord.begin(), c.ord.end(), 0);
  std::stable_sort(c.ord.begin(), c.ord.end(),
                   [&](int a, int d) { return std::abs(c.theta[a]) > std::abs(c.theta[d]); });
  int pos = std::min(nev, k);
  while (pos < k && std::abs(std::abs(c.theta[c.ord[pos]]) - std::abs(c.theta[c.ord[pos - 1]])) <=
                        1e-9 * std::abs(c.theta[c.ord[pos - 1]]))
    ++pos;
  c.nw = pos;
  c.wanted.assign(c.ord.begin(), c.ord.begin() + c.nw);
  // Ritz vectors of the wanted values in the Schur basis (y = Q x) and
  // residual estimates ||E y|| = ||(E Q) x|| (E = rows k..k+b of H)
  c.k = k;
  c.Y.clear();
  schur_eigvecs_real(k, c.TR, c.QR, c.theta, c.X, 1e-11, &c.wanted, true);
  std::vector<double> EQ((size_t)b * k, 0.0);
  for (int col = 0; col < k; ++col)
    for (int r = 0; r < b; ++r) {
      double s = 0.0;
      for (int t2 = 0; t2 < k; ++t2) s += Hat(k + r, t2) * c.QR[t2 + (size_t)col * k];
      EQ[r + (size_t)col * b] = s;
    }
  c.nconv = 0;
  c.tol = tol;
  c.conv.assign(k, 0);
  for (int p = 0; p < c.nw; ++p) {
    const int i = c.ord[p];
    double s = 0.0;
    for (int r = 0; r < b; ++r) {
      cplx acc = 0.0;
      for (int col = 0; col < k; ++col) acc += EQ[r + (size_t)col * b] * c.X[col + (size_t)i * k];
      s += std::norm(acc);
    }
    if (std::sqrt(s) <= tol * std::abs(c.theta[i])) {
      ++c.nconv;
      c.conv[i] = 1;
    }
  }
  return 0;
}

void ks_ritz_vectors(KsCycle& c) {
  const int k = c.k;
  c.Y.assign((size_t)k * k, cplx(0.0));
  for (int i : c.wanted) {
    const cplx* x = &c.X[(size_t)i * k];
    cplx* y = &c.Y[(size_t)i * k];
    for (int j = 0; j < k; ++j) {
      if (x[j] == cplx(0.0)) continue;
      const double* q = &c.QR[(size_t)j * k];
      for (int r = 0; r < k; ++r) y[r] += q[r] * x[j];
    }
  }
}

void ks_restart(const std::vector<double>& H, int ldh, int k, int b, int m, int nev, int keep, KsCycle& c) {
  auto Hat = [&](int r, int col) { return H[r + (size_t)col * ldh]; };
  auto same = [&](int p) {  // ord[p] continues the |theta| cluster of ord[p-1]
    return std::abs(std::abs(c.theta[c.ord[p]]) - std::abs(c.theta[c.ord[p - 1]])) <=
           1e-9 * std::abs(c.theta[c.ord[p - 1]]);
  };
  int kk = keep > 0 ? std::max(keep, nev) : nev + (k - nev) / 2;
  kk = std::min(kk, m - b);
  kk = std::max(kk, std::min(c.nw, m - b));
  int kend = std::max(1, kk);
  while (kend < k && same(kend)) ++kend;
  if (kend + b <= m) {
    kk = kend;
  } else {  // step back to a cluster boundary
    while (kk > 1 && same(kk)) --kk;
  }
  std::vector<char> kept(k, 0);
  for (int p = 0; p < kk; ++p) kept[c.ord[p]] = 1;
  const int kin = k + b;
  // Preferred: reorder the real Schur form.  The leading r columns of its
  // vectors are then a real orthonormal basis of the kept invariant subspace
  // and the new projected matrix is [T_rr; E Q_r].
  c.nlock = 0;
  {
    std::vector<double> TR = c.TR, QR = c.QR;
    // converged kept values first (a pair counts only if both halves passed)
    std::vector<int> bst, bsz;
    for (int i = 0; i < k;) {
      const int sz = (i + 1 < k && TR[(i + 1) + (size_t)i * k] != 0.0) ? 2 : 1;
      bst.push_back(i);
      bsz.push_back(sz);
      i += sz;
    }
    std::vector<char> lock(k, 0), kept2 = kept;
    int nl = 0;
    for (size_t q = 0; q < bst.size(); ++q) {
      bool all = true;
      for (int u = 0; u < bsz[q]; ++u) all = all && kept[bst[q] + u] && (int)c.conv.size() == k && c.conv[bst[q] + u];
      if (all)
        for (int u = 0; u < bsz[q]; ++u) lock[bst[q] + u] = 1;
      nl += all ? bsz[q] : 0;
    }
    if (nl > 0 && schur_select_real(k, TR, QR, lock) == nl) {
      // the selection is stable: locked blocks in their order, then the rest
      int pos = 0;
      for (int pass = 0; pass < 2; ++pass)
        for (size_t q = 0; q < bst.size(); ++q)
          if ((lock[bst[q]] != 0) == (pass == 0))
            for (int u = 0; u < bsz[q]; ++u) kept2[pos++] = kept[bst[q] + u];
    } else {
      TR = c.TR;
      QR = c.QR;
      nl = 0;
    }
    const int r = schur_select_real(k, TR, QR, kept2);
    if (r > 0) {
      c.Hn.assign((size_t)ldh * ldh, 0.0);
      for (int col = 0; col < r; ++col) {
        for (int rr = 0; rr <= std::min(col + 1, r - 1); ++rr) c.Hn[rr + (size_t)col * ldh] = TR[rr + (size_t)col * k];
        for (int rr = 0; rr < b; ++rr) {
          double s = 0.0;
          for (int t2 = 0; t2 < k; ++t2) s += Hat(k + rr, t2) * QR[t2 + (size_t)col * k];
          c.Hn[r + rr + (size_t)col * ldh] = s;
        }
      }
      // locking: the leading run of converged blocks whose columns of E Q are
      // at most tol |theta| (|theta|^2 = the block's determinant for a pair)
      int nlock = 0;
      for (int i = 0; i < std::min(nl, r);) {
        const int sz = (i + 1 < r && c.Hn[(i + 1) + (size_t)i * ldh] != 0.0) ? 2 : 1;
        const double* t0 = &c.Hn[(size_t)i * ldh];
        const double th = sz == 1 ? std::abs(t0[i])
                                  : std::sqrt(std::abs(t0[i] * t0[i + 1 + ldh] - t0[i + ldh] * t0[i + 1]));
        bool small = i + sz <= nl;
        for (int u = 0; u < sz && small; ++u) {
          double e2 = 0.0;
          for (int rr = 0; rr < b; ++rr) e2 += c.Hn[r + rr + (size_t)(i + u) * ldh] * c.Hn[r + rr + (size_t)(i + u) * ldh];
          small = std::sqrt(e2) <= c.tol * th;
        }
        if (!small) break;
        i += sz;
        nlock = i;
      }
      for (int col = 0; col < nlock; ++col)
        for (int rr = 0; rr < b; ++rr) c.Hn[r + rr + (size_t)col * ldh] = 0.0;
      c.nlock = nlock;
      const int kout = r + b;
      c.Qe.assign((size_t)kin * kout, 0.0);
      for (int col = 0; col < r; ++col)
        for (int t2 = 0; t2 < k; ++t2) c.Qe[t2 + (size_t)col * kin] = QR[t2 + (size_t)col * k];
      for (int q = 0; q < b; ++q) c.Qe[(k + q) + (size_t)(r + q) * kin] = 1.0;
      c.r = r;
      c.real_restart = true;
      return;
    }
  }
  // Fallback (an ill-conditioned exchange): reorder the complex Schur form and
  // take a real basis of the kept span.
  c.real_restart = false;
  if (c.T.empty()) schur_complexify(k, c.TR, c.QR, c.T, c.Z);
  std::vector<cplx> T = c.T, Z = c.Z;
  schur_select(k, T, Z, kept);
  std::vector<double> Qk;
  const int r = realify(k, kk, Z, Qk);
  std::vector<double> Hk((size_t)k * k);
  for (int col = 0; col < k; ++col)
    for (int rr = 0; rr < k; ++rr) Hk[rr + (size_t)col * k] = Hat(rr, col);
  // T_new = Qk^T H_k Qk, E_new = E Qk
  std::vector<double> HQ((size_t)k * r, 0.0);
  for (int col = 0; col < r; ++col)
    for (int t2 = 0; t2 < k; ++t2) {
      const double q = Qk[t2 + (size_t)col * k];
      if (q == 0.0) continue;
      for (int rr = 0; rr < k; ++rr) HQ[rr + (size_t)col * k] += Hk[rr + (size_t)t2 * k] * q;
    }
  c.Hn.assign((size_t)ldh * ldh, 0.0);
  for (int col = 0; col < r; ++col) {
    for (int rr = 0; rr < r; ++rr) {
      double s = 0.0;
      for (int t2 = 0; t2 < k; ++t2) s += Qk[t2 + (size_t)rr * k] * HQ[t2 + (size_t)col * k];
      c.Hn[rr + (size_t)col * ldh] = s;
    }
    for (int rr = 0; rr < b; ++rr) {
      double s = 0.0;
      for (int t2 = 0; t2 < k; ++t2) s += Hat(k + rr, t2) * Qk[t2 + (size_t)col * k];
      c.Hn[r + rr + (size_t)col * ldh] = s;
    }
  }
  // V_new = [V_k Qk, V_{k:k+b}]
  const int kout = r + b;
  c.Qe.assign((size_t)kin * kout, 0.0);
  for (int col = 0; col < r; ++col)
    for (int t2 = 0; t2 < k; ++t2) c.Qe[t2 + (size_t)col * kin] = Qk[t2 + (size_t)col * k];
  for (int q = 0; q < b; ++q) c.Qe[(k + q) + (size_t)(r + q) * kin] = 1.0;
  c.r = r;
}

PairForms pair_forms(const double f[11]) {
  PairForms pf;
  // unconjugated forms u^T A u = a^T A a - b^T A b + 2i a^T A b
  pf.qm = cplx(f[0] - f[1], 2 * f[2]);
  pf.qc = cplx(f[3] - f[4], 2 * f[5]);
  pf.qk = cplx(f[6] - f[7], 2 * f[8]);
  pf.uMu = f[0] + f[1];
  pf.unorm2 = f[9] + f[10];
  return pf;
}

cplx rayleigh_polish(const PairForms& pf, cplx ritz) {
  const cplx disc = std::sqrt(pf.qc * pf.qc - 4.0 * pf.qm * pf.qk);
  const cplx r1 = (-pf.qc + disc) / (2.0 * pf.qm), r2 = (-pf.qc - disc) / (2.0 * pf.qm);
  const cplx pick = std::abs(r1 - ritz) < std::abs(r2 - ritz) ? r1 : r2;
  return (std::isfinite(pick.real()) && std::isfinite(pick.imag())) ? pick : ritz;
}

double scaled_residual(double resid2, cplx lam, const double norms[3], double unorm2) {
  const double al = std::abs(lam);
  return std::sqrt(resid2) / ((al * al * norms[2] + al * norms[1] + norms[0]) * std::sqrt(unorm2));
}

}  // namespace riga
