// Small dense eigensolver for the projected Krylov matrix (host).
#include "small_eig.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace riga {

namespace {

inline double abs1(cplx z) { return std::abs(z.real()) + std::abs(z.imag()); }

// Givens rotation G = [[c, s], [-conj(s), c]] with c real and G [x; y] = [r; 0].
inline void givens(cplx x, cplx y, double& c, cplx& s) {
  if (y == cplx(0.0)) { c = 1.0; s = 0.0; return; }
  if (x == cplx(0.0)) { c = 0.0; s = 1.0; return; }
  double nx = std::abs(x), nrm = std::hypot(nx, std::abs(y));
  c = nx / nrm;
  s = (x / nx) * std::conj(y) / nrm;
}

// Real Householder reduction to upper Hessenberg form: A = Q H Q^T.
void hessenberg(int n, std::vector<double>& H, std::vector<double>& Q) {
  auto h = [&](int i, int j) -> double& { return H[i + (size_t)j * n]; };
  auto q = [&](int i, int j) -> double& { return Q[i + (size_t)j * n]; };
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) q(i, i) = 1.0;
  std::vector<double> v(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += h(i, k) * h(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (h(k + 1, k) > 0) alpha = -alpha;
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) { v[i] = h(i, k); }
    v[k + 1] -= alpha;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // rows k+1..n-1: H -= beta v (v^T H)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * h(i, j);
      s *= beta;
      for (int i = k + 1; i < n; ++i) h(i, j) -= s * v[i];
    }
    // columns k+1..n-1: H -= beta (H v) v^T, and the same for Q
    for (int i = 0; i < n; ++i) {
      double s = 0.0, t = 0.0;
      for (int j = k + 1; j < n; ++j) { s += h(i, j) * v[j]; t += q(i, j) * v[j]; }
      s *= beta; t *= beta;
      for (int j = k + 1; j < n; ++j) { h(i, j) -= s * v[j]; q(i, j) -= t * v[j]; }
    }
    for (int i = k + 2; i < n; ++i) h(i, k) = 0.0;
  }
}

}  // namespace

int schur_complex(int n, const double* A, std::vector<cplx>& T, std::vector<cplx>& Z) {
  std::vector<double> H(A, A + (size_t)n * n), Q;
  hessenberg(n, H, Q);
  T.assign((size_t)n * n, cplx(0.0));
  Z.assign((size_t)n * n, cplx(0.0));
  for (size_t k = 0; k < (size_t)n * n; ++k) { T[k] = H[k]; Z[k] = Q[k]; }
  auto t = [&](int i, int j) -> cplx& { return T[i + (size_t)j * n]; };
  auto z = [&](int i, int j) -> cplx& { return Z[i + (size_t)j * n]; };
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) anorm = std::max(anorm, abs1(t(i, j)));
  if (anorm == 0.0) return 0;
  int hi = n - 1, iter = 0, total = 0;
  const int maxtotal = 100 * std::max(n, 10);
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      double s = abs1(t(l - 1, l - 1)) + abs1(t(l, l));
      if (s == 0.0) s = anorm;
      if (abs1(t(l, l - 1)) <= eps * s) { t(l, l - 1) = 0.0; break; }
      --l;
    }
    if (l == hi) { --hi; iter = 0; continue; }
    if (++total > maxtotal) return -1;
    ++iter;
    cplx mu;
    if (iter % 11 == 10) {
      // exceptional shift to break a possible cycle
      mu = t(hi, hi) + 0.75 * std::abs(t(hi, hi - 1).real()) + cplx(0.0, 0.43 * std::abs(t(hi, hi - 1)));
    } else {
      cplx a = t(hi - 1, hi - 1), b = t(hi - 1, hi), c = t(hi, hi - 1), d = t(hi, hi);
      cplx half = 0.5 * (a - d);
      cplx disc = std::sqrt(half * half + b * c);
      cplx m1 = d - (b * c) / (half + disc), m2 = d - (b * c) / (half - disc);
      if (half + disc == cplx(0.0)) m1 = d;
      if (half - disc == cplx(0.0)) m2 = d;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    cplx x = t(l, l) - mu, y = t(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) { x = t(k, k - 1); y = t(k + 1, k - 1); }
      double c; cplx s;
      givens(x, y, c, s);
      for (int j = (k > l ? k - 1 : l); j < n; ++j) {
        cplx t1 = t(k, j), t2 = t(k + 1, j);
        t(k, j) = c * t1 + s * t2;
        t(k + 1, j) = -std::conj(s) * t1 + c * t2;
      }
      if (k > l) t(k + 1, k - 1) = 0.0;
      const int imax = std::min(k + 2, hi);
      for (int i = 0; i <= imax; ++i) {
        cplx t1 = t(i, k), t2 = t(i, k + 1);
        t(i, k) = c * t1 + std::conj(s) * t2;
        t(i, k + 1) = -s * t1 + c * t2;
      }
      for (int i = 0; i < n; ++i) {
        cplx t1 = z(i, k), t2 = z(i, k + 1);
        z(i, k) = c * t1 + std::conj(s) * t2;
        z(i, k + 1) = -s * t1 + c * t2;
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) t(i, j) = 0.0;
  return 0;
}

namespace {

// Exchange the adjacent diagonal entries k and k+1 of the triangular T.
void swap_adjacent(int n, std::vector<cplx>& T, std::vector<cplx>& Z, int k) {
  auto t = [&](int i, int j) -> cplx& { return T[i + (size_t)j * n]; };
  auto z = [&](int i, int j) -> cplx& { return Z[i + (size_t)j * n]; };
  cplx t11 = t(k, k), t22 = t(k + 1, k + 1), t12 = t(k, k + 1);
  if (t11 == t22) return;
  // [t12; t22 - t11] is the eigenvector of t22; rotate it onto e_1
  double c; cplx s;
  givens(t12, t22 - t11, c, s);
  for (int j = k; j < n; ++j) {
    cplx a = t(k, j), b = t(k + 1, j);
    t(k, j) = c * a + s * b;
    t(k + 1, j) = -std::conj(s) * a + c * b;
  }
  for (int i = 0; i <= k + 1; ++i) {
    cplx a = t(i, k), b = t(i, k + 1);
    t(i, k) = c * a + std::conj(s) * b;
    t(i, k + 1) = -s * a + c * b;
  }
  for (int i = 0; i < n; ++i) {
    cplx a = z(i, k), b = z(i, k + 1);
    z(i, k) = c * a + std::conj(s) * b;
    z(i, k + 1) = -s * a + c * b;
  }
  t(k + 1, k) = 0.0;
  t(k, k) = t22;
  t(k + 1, k + 1) = t11;
}

}  // namespace

void schur_reorder(int n, std::vector<cplx>& T, std::vector<cplx>& Z, const std::vector<int>& order) {
  // position of each original diagonal entry as swaps proceed
  std::vector<int> where(n), who(n);
  for (int i = 0; i < n; ++i) { where[i] = i; who[i] = i; }
  for (size_t dst = 0; dst < order.size(); ++dst) {
    int cur = where[order[dst]];
    for (int k = cur - 1; k >= (int)dst; --k) {
      swap_adjacent(n, T, Z, k);
      int a = who[k], b = who[k + 1];
      who[k] = b; who[k + 1] = a;
      where[b] = k; where[a] = k + 1;
    }
  }
}

void schur_eigvecs(int n, const std::vector<cplx>& T, const std::vector<cplx>& Z,
                   std::vector<cplx>& Y, double cluster_tol) {
  auto t = [&](int i, int j) { return T[i + (size_t)j * n]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(t(i, i)));
  if (scale == 0.0) scale = 1.0;
  const double tiny = std::numeric_limits<double>::min() / std::numeric_limits<double>::epsilon();
  Y.assign((size_t)n * n, cplx(0.0));
  std::vector<cplx> x(n);
  for (int k = 0; k < n; ++k) {
    const cplx lam = t(k, k);
    std::fill(x.begin(), x.end(), cplx(0.0));
    x[k] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      cplx s = 0.0;
      for (int j = i + 1; j <= k; ++j) s += t(i, j) * x[j];
      cplx d = t(i, i) - lam;
      if (std::abs(d) <= cluster_tol * scale) {
        x[i] = 0.0;
      } else {
        if (std::abs(d) < tiny) d = tiny;
        x[i] = -s / d;
      }
    }
    double nrm = 0.0;
    cplx* y = &Y[(size_t)k * n];
    for (int i = 0; i < n; ++i) {
      cplx acc = 0.0;
      for (int j = 0; j <= k; ++j) acc += Z[i + (size_t)j * n] * x[j];
      y[i] = acc;
      nrm += std::norm(acc);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) y[i] /= nrm;
  }
}

int realify(int n, int k, const std::vector<cplx>& Z, std::vector<double>& Q) {
  const int m = 2 * k;
  std::vector<double> A((size_t)n * m);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < n; ++i) {
      A[i + (size_t)j * n] = Z[i + (size_t)j * n].real();
      A[i + (size_t)(k + j) * n] = Z[i + (size_t)j * n].imag();
    }
  // Householder QR with column pivoting
  std::vector<int> perm(m);
  for (int j = 0; j < m; ++j) perm[j] = j;
  std::vector<std::vector<double>> vs;
  std::vector<double> betas;
  double r00 = 0.0;
  int rank = 0;
  const int steps = std::min(n, m);
  for (int j = 0; j < steps; ++j) {
    int best = j;
    double bn = -1.0;
    for (int c = j; c < m; ++c) {
      double s = 0.0;
      for (int i = j; i < n; ++i) s += A[i + (size_t)c * n] * A[i + (size_t)c * n];
      if (s > bn) { bn = s; best = c; }
    }
    const double cn = std::sqrt(std::max(bn, 0.0));
    if (j == 0) r00 = cn;
    if (cn <= 1e-9 * r00 || cn == 0.0) break;
    if (best != j) {
      for (int i = 0; i < n; ++i) std::swap(A[i + (size_t)j * n], A[i + (size_t)best * n]);
      std::swap(perm[j], perm[best]);
    }
    std::vector<double> v(n, 0.0);
    double alpha = cn;
    if (A[j + (size_t)j * n] > 0) alpha = -alpha;
    for (int i = j; i < n; ++i) v[i] = A[i + (size_t)j * n];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < n; ++i) vv += v[i] * v[i];
    double beta = vv > 0 ? 2.0 / vv : 0.0;
    for (int c = j; c < m; ++c) {
      double s = 0.0;
      for (int i = j; i < n; ++i) s += v[i] * A[i + (size_t)c * n];
      s *= beta;
      for (int i = j; i < n; ++i) A[i + (size_t)c * n] -= s * v[i];
    }
    vs.push_back(v);
    betas.push_back(beta);
    ++rank;
  }
  // explicit Q = H_0 H_1 ... H_{r-1} applied to the first r unit vectors
  Q.assign((size_t)n * rank, 0.0);
  for (int c = 0; c < rank; ++c) Q[c + (size_t)c * n] = 1.0;
  for (int j = rank - 1; j >= 0; --j) {
    const std::vector<double>& v = vs[j];
    for (int c = 0; c < rank; ++c) {
      double s = 0.0;
      for (int i = j; i < n; ++i) s += v[i] * Q[i + (size_t)c * n];
      s *= betas[j];
      for (int i = j; i < n; ++i) Q[i + (size_t)c * n] -= s * v[i];
    }
  }
  return rank;
}

}  // namespace riga
