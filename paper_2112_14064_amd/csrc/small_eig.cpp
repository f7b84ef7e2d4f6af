// Small dense eigensolver for the projected Krylov matrix (host).
#include "small_eig.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

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

// Column kernels of the reductions below; the arguments never overlap, so the
// loops vectorise.
inline double dot(int len, const double* __restrict__ a, const double* __restrict__ b) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 3 < len; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < len; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

inline void axpy(int len, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int i = 0; i < len; ++i) y[i] += a * x[i];
}

// Real Householder reduction to upper Hessenberg form: A = Q H Q^T.
void hessenberg(int n, std::vector<double>& H, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
  double* h = H.data();
  double* q = Q.data();
  std::vector<double> v(n), w(n), z(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;               // length of the reflector (rows k+1..n-1)
    double* hk = h + (size_t)k * n + k + 1;
    const double alpha0 = std::sqrt(dot(m, hk, hk));
    if (alpha0 == 0.0) continue;
    const double alpha = hk[0] > 0 ? -alpha0 : alpha0;
    double* vk = v.data() + k + 1;
    for (int i = 0; i < m; ++i) vk[i] = hk[i];
    vk[0] -= alpha;
    const double vv = dot(m, vk, vk);
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // rows k+1..n-1: H -= beta v (v^T H) (columns before k are already reduced)
    for (int j = k; j < n; ++j) {
      double* hj = h + (size_t)j * n + k + 1;
      axpy(m, -beta * dot(m, vk, hj), vk, hj);
    }
    // columns k+1..n-1: H -= beta (H v) v^T, and the same for Q; both by
    // whole columns (w = H v, z = Q v first)
    std::fill(w.begin(), w.end(), 0.0);
    std::fill(z.begin(), z.end(), 0.0);
    for (int j = k + 1; j < n; ++j) {
      axpy(n, v[j], h + (size_t)j * n, w.data());
      axpy(n, v[j], q + (size_t)j * n, z.data());
    }
    for (int j = k + 1; j < n; ++j) {
      axpy(n, -beta * v[j], w.data(), h + (size_t)j * n);
      axpy(n, -beta * v[j], z.data(), q + (size_t)j * n);
    }
    for (int i = k + 2; i < n; ++i) h[i + (size_t)k * n] = 0.0;
  }
}

}  // namespace

namespace {

// Householder vector of a 2- or 3-vector: (I - beta v v^T) x = alpha e_1 with
// v[0] = 1; returns false (identity) for x = 0.
inline bool house(int m, const double* x, double* v, double& beta) {
  double nrm = 0.0;
  for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
  nrm = std::sqrt(nrm);
  if (nrm == 0.0) return false;
  const double alpha = x[0] > 0 ? -nrm : nrm;
  const double v0 = x[0] - alpha;
  v[0] = 1.0;
  double vv = 1.0;
  for (int i = 1; i < m; ++i) { v[i] = x[i] / v0; vv += v[i] * v[i]; }
  beta = 2.0 / vv;
  return true;
}

// Reflection (I - beta v v^T), v = (1, v1, v2), applied from the right to
// rows 0..len-1 of three columns.
inline void refl3(int len, double* __restrict__ a, double* __restrict__ b, double* __restrict__ c, double beta,
                  double v1, double v2) {
  for (int r = 0; r < len; ++r) {
    const double t = beta * (a[r] + v1 * b[r] + v2 * c[r]);
    a[r] -= t;
    b[r] -= t * v1;
    c[r] -= t * v2;
  }
}

inline void refl2(int len, double* __restrict__ a, double* __restrict__ b, double beta, double v1) {
  for (int r = 0; r < len; ++r) {
    const double t = beta * (a[r] + v1 * b[r]);
    a[r] -= t;
    b[r] -= t * v1;
  }
}

// Real Schur form H = Q T Q^T of an upper Hessenberg H by Francis double-shift
// QR steps with deflation (the implicit double-shift algorithm in the form
// of Golub and Van Loan, Alg. 7.5.1-7.5.2), accumulating into Q.  T is quasi
// upper triangular: 1x1 blocks and 2x2 blocks (subdiagonal nonzero).
int real_schur(int n, std::vector<double>& H, std::vector<double>& Q) {
  auto h = [&](int i, int j) -> double& { return H[i + (size_t)j * n]; };
  auto q = [&](int i, int j) -> double& { return Q[i + (size_t)j * n]; };
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j + 1, n - 1); ++i) anorm = std::max(anorm, std::abs(h(i, j)));
  if (anorm == 0.0) return 0;
  int i = n - 1, its = 0, total = 0;
  const int maxtotal = 60 * std::max(n, 10);
  while (i >= 0) {
    // deflation point: the last negligible subdiagonal entry above row i
    int l = i;
    while (l > 0) {
      double sc = std::abs(h(l - 1, l - 1)) + std::abs(h(l, l));
      if (sc == 0.0) sc = anorm;
      if (std::abs(h(l, l - 1)) <= eps * sc) { h(l, l - 1) = 0.0; break; }
      --l;
    }
    if (l == i) { --i; its = 0; continue; }          // 1x1 block
    if (l == i - 1) { i -= 2; its = 0; continue; }   // 2x2 block
    if (++total > maxtotal) return -1;
    ++its;
    // shifts: eigenvalues of the trailing 2x2 block (trace s, determinant t),
    // replaced by ad hoc values at iterations 10 and 20 to break cycles
    double sh, th;
    if (its == 10 || its == 20) {
      const double w = std::abs(h(i, i - 1)) + std::abs(h(i - 1, i - 2));
      sh = 1.5 * w;
      th = w * w;
    } else {
      sh = h(i - 1, i - 1) + h(i, i);
      th = h(i - 1, i - 1) * h(i, i) - h(i - 1, i) * h(i, i - 1);
    }
    // first column of (H - s1)(H - s2) on the active block [l, i]
    double x[3];
    x[0] = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - sh * h(l, l) + th;
    x[1] = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - sh);
    x[2] = h(l + 1, l) * h(l + 2, l + 1);
    const int nw = i - l + 1;
    double v[3], beta;
    for (int k = 0; k <= nw - 3; ++k) {
      const int r0 = l + k;
      if (house(3, x, v, beta)) {
        const int c0 = (k == 0) ? l : r0 - 1;
        for (int j = c0; j < n; ++j) {
          const double sdot = beta * (h(r0, j) + v[1] * h(r0 + 1, j) + v[2] * h(r0 + 2, j));
          h(r0, j) -= sdot;
          h(r0 + 1, j) -= sdot * v[1];
          h(r0 + 2, j) -= sdot * v[2];
        }
        const int rmax = std::min(r0 + 3, i);
        refl3(rmax + 1, &h(0, r0), &h(0, r0 + 1), &h(0, r0 + 2), beta, v[1], v[2]);
        refl3(n, &q(0, r0), &q(0, r0 + 1), &q(0, r0 + 2), beta, v[1], v[2]);
      }
      if (k > 0) h(r0 + 1, r0 - 1) = h(r0 + 2, r0 - 1) = 0.0;   // the bulge moved on
      x[0] = h(r0 + 1, r0);
      x[1] = h(r0 + 2, r0);
      if (k < nw - 3) x[2] = h(r0 + 3, r0);
    }
    // last 2-vector reflection on rows / columns i-1, i
    if (house(2, x, v, beta)) {
      for (int j = i - 2; j < n; ++j) {
        const double sdot = beta * (h(i - 1, j) + v[1] * h(i, j));
        h(i - 1, j) -= sdot;
        h(i, j) -= sdot * v[1];
      }
      refl2(i + 1, &h(0, i - 1), &h(0, i), beta, v[1]);
      refl2(n, &q(0, i - 1), &q(0, i), beta, v[1]);
    }
    h(i, i - 2) = 0.0;
  }
  return 0;
}

}  // namespace

int schur_real(int n, const double* A, std::vector<double>& T, std::vector<double>& Q) {
  T.assign(A, A + (size_t)n * n);
  hessenberg(n, T, Q);
  if (real_schur(n, T, Q) != 0) return -1;
  for (int j = 0; j < n; ++j)
    for (int i = j + 2; i < n; ++i) T[i + (size_t)j * n] = 0.0;
  return 0;
}

void schur_complexify(int n, const std::vector<double>& TR, const std::vector<double>& QR, std::vector<cplx>& T,
                      std::vector<cplx>& Z) {
  T.assign((size_t)n * n, cplx(0.0));
  Z.assign((size_t)n * n, cplx(0.0));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j + 1, n - 1); ++i) T[i + (size_t)j * n] = TR[i + (size_t)j * n];
  for (size_t k = 0; k < (size_t)n * n; ++k) Z[k] = QR[k];
  auto t = [&](int i, int j) -> cplx& { return T[i + (size_t)j * n]; };
  auto z = [&](int i, int j) -> cplx& { return Z[i + (size_t)j * n]; };
  // complex Schur form: triangularise every 2x2 block with the unitary whose
  // first column is an eigenvector of the block
  for (int k = 0; k + 1 < n; ++k) {
    if (t(k + 1, k) == cplx(0.0)) continue;
    const cplx a = t(k, k), b = t(k, k + 1), c = t(k + 1, k), d = t(k + 1, k + 1);
    const cplx half = 0.5 * (a - d);
    const cplx disc = std::sqrt(half * half + b * c);
    const cplx lam = 0.5 * (a + d) + disc;
    // eigenvector of [[a, b], [c, d]] for lam: [b; lam - a] or [lam - d; c]
    cplx v1 = b, v2 = lam - a;
    if (std::abs(v1) + std::abs(v2) < std::abs(lam - d) + std::abs(c)) { v1 = lam - d; v2 = c; }
    const double nv = std::sqrt(std::norm(v1) + std::norm(v2));
    v1 /= nv; v2 /= nv;
    // G = [v, w] with w = [-conj(v2); conj(v1)]; T <- G^H T G, Z <- Z G
    for (int j = k; j < n; ++j) {
      const cplx t1 = t(k, j), t2 = t(k + 1, j);
      t(k, j) = std::conj(v1) * t1 + std::conj(v2) * t2;
      t(k + 1, j) = -v2 * t1 + v1 * t2;
    }
    for (int r = 0; r <= k + 1; ++r) {
      const cplx t1 = t(r, k), t2 = t(r, k + 1);
      t(r, k) = t1 * v1 + t2 * v2;
      t(r, k + 1) = -t1 * std::conj(v2) + t2 * std::conj(v1);
    }
    for (int r = 0; r < n; ++r) {
      const cplx t1 = z(r, k), t2 = z(r, k + 1);
      z(r, k) = t1 * v1 + t2 * v2;
      z(r, k + 1) = -t1 * std::conj(v2) + t2 * std::conj(v1);
    }
    t(k + 1, k) = 0.0;
    ++k;   // the next block starts after this one
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) t(i, j) = 0.0;
}

int schur_complex(int n, const double* A, std::vector<cplx>& T, std::vector<cplx>& Z) {
  std::vector<double> TR, QR;
  if (schur_real(n, A, TR, QR) != 0) return -1;
  schur_complexify(n, TR, QR, T, Z);
  return 0;
}

namespace {

// Exchange of the adjacent diagonal blocks A11 (p x p, at row j) and A22
// (q x q) of a real quasi-triangular T, p, q in {1, 2}, by the direct method
// of Bai and Demmel (1993): X with A11 X - X A22 = A12 spans, with the
// identity below it, the invariant subspace of A22; an orthogonal U whose
// first q columns span [-X; I] moves A22's eigenvalues to the top.
// Returns false when the Sylvester equation is (nearly) singular or the
// block left below the exchanged pair is not negligible; T and Q are then
// partly updated and must be discarded.
bool swap_blocks(int n, std::vector<double>& T, std::vector<double>& Q, int j, int p, int q) {
  auto t = [&](int i, int c) -> double& { return T[i + (size_t)c * n]; };
  const int w = p + q;
  const double eps = std::numeric_limits<double>::epsilon();
  double wnorm = 0.0;
  for (int c = j; c < j + w; ++c)
    for (int i = j; i < j + w; ++i) wnorm = std::max(wnorm, std::abs(t(i, c)));
  // Kronecker system (I_q (x) A11 - A22^T (x) I_p) vec(X) = vec(A12), unknown X[a + p b]
  const int m = p * q;
  double M[4][5] = {{0}};
  for (int b = 0; b < q; ++b)
    for (int a = 0; a < p; ++a) {
      const int row = a + p * b;
      for (int c = 0; c < p; ++c) M[row][c + p * b] += t(j + a, j + c);
      for (int d = 0; d < q; ++d) M[row][a + p * d] -= t(j + p + d, j + p + b);
      M[row][m] = t(j + a, j + p + b);
    }
  // Gaussian elimination with complete pivoting
  int colp[4] = {0, 1, 2, 3};
  for (int k = 0; k < m; ++k) {
    int br = k, bc = k;
    double best = -1.0;
    for (int r = k; r < m; ++r)
      for (int c = k; c < m; ++c)
        if (std::abs(M[r][c]) > best) { best = std::abs(M[r][c]); br = r; bc = c; }
    if (best <= eps * std::max(wnorm, std::numeric_limits<double>::min())) return false;
    for (int c = 0; c <= m; ++c) std::swap(M[k][c], M[br][c]);
    for (int r = 0; r < m; ++r) std::swap(M[r][k], M[r][bc]);
    std::swap(colp[k], colp[bc]);
    for (int r = k + 1; r < m; ++r) {
      const double f = M[r][k] / M[k][k];
      for (int c = k; c <= m; ++c) M[r][c] -= f * M[k][c];
    }
  }
  double y[4], X[4];
  for (int k = m - 1; k >= 0; --k) {
    double s = M[k][m];
    for (int c = k + 1; c < m; ++c) s -= M[k][c] * y[c];
    y[k] = s / M[k][k];
  }
  for (int k = 0; k < m; ++k) X[colp[k]] = y[k];
  // Householder QR of W = [-X; I_q] (w x q): reflectors (I - beta v v^T)
  double W[4][2] = {{0}};
  for (int b = 0; b < q; ++b) {
    for (int a = 0; a < p; ++a) W[a][b] = -X[a + p * b];
    W[p + b][b] = 1.0;
  }
  double V[2][4] = {{0}}, beta[2] = {0, 0};
  for (int k = 0; k < q; ++k) {
    double nrm = 0.0;
    for (int i = k; i < w; ++i) nrm += W[i][k] * W[i][k];
    nrm = std::sqrt(nrm);
    const double alpha = W[k][k] > 0 ? -nrm : nrm;
    for (int i = 0; i < w; ++i) V[k][i] = (i < k) ? 0.0 : W[i][k];
    V[k][k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < w; ++i) vv += V[k][i] * V[k][i];
    beta[k] = vv > 0.0 ? 2.0 / vv : 0.0;
    for (int c = k; c < q; ++c) {
      double sd = 0.0;
      for (int i = k; i < w; ++i) sd += V[k][i] * W[i][c];
      sd *= beta[k];
      for (int i = k; i < w; ++i) W[i][c] -= sd * V[k][i];
    }
  }
  // T <- U^T T U and Q <- Q U with U = H_0 H_1 (window rows / columns j .. j+w-1)
  for (int k = 0; k < q; ++k) {
    const double* v = V[k];
    for (int c = j; c < n; ++c) {
      double sd = 0.0;
      for (int i = 0; i < w; ++i) sd += v[i] * t(j + i, c);
      sd *= beta[k];
      for (int i = 0; i < w; ++i) t(j + i, c) -= sd * v[i];
    }
    for (int r = 0; r < j + w; ++r) {
      double sd = 0.0;
      for (int i = 0; i < w; ++i) sd += t(r, j + i) * v[i];
      sd *= beta[k];
      for (int i = 0; i < w; ++i) t(r, j + i) -= sd * v[i];
    }
    for (int r = 0; r < n; ++r) {
      double sd = 0.0;
      for (int i = 0; i < w; ++i) sd += Q[r + (size_t)(j + i) * n] * v[i];
      sd *= beta[k];
      for (int i = 0; i < w; ++i) Q[r + (size_t)(j + i) * n] -= sd * v[i];
    }
  }
  // the p x q block below the new leading q x q block must be negligible
  double low = 0.0;
  for (int c = j; c < j + q; ++c)
    for (int i = j + q; i < j + w; ++i) low = std::max(low, std::abs(t(i, c)));
  if (low > 10.0 * eps * std::max(wnorm, 1.0)) return false;
  for (int c = j; c < j + q; ++c)
    for (int i = j + q; i < j + w; ++i) t(i, c) = 0.0;
  return true;
}

}  // namespace

int schur_select_real(int n, std::vector<double>& T, std::vector<double>& Q, const std::vector<char>& keep) {
  // blocks of the quasi-triangular form: start, size, kept
  std::vector<int> bs, bz;
  std::vector<char> bk;
  for (int i = 0; i < n;) {
    const int sz = (i + 1 < n && T[(i + 1) + (size_t)i * n] != 0.0) ? 2 : 1;
    if (sz == 2 && keep[i] != keep[i + 1]) return -1;   // a conjugate pair is kept whole
    bs.push_back(i); bz.push_back(sz); bk.push_back(keep[i] != 0);
    i += sz;
  }
  // walk up from the bottom; every block not kept sinks to the end of the kept ones
  const int nb = (int)bs.size();
  int end = nb;
  for (int b = nb - 1; b >= 0; --b) {
    if (bk[b]) continue;
    for (int k = b; k < end - 1; ++k) {
      // blocks k (not kept) and k+1 (kept) exchange places
      if (!swap_blocks(n, T, Q, bs[k], bz[k], bz[k + 1])) return -1;
      bs[k + 1] = bs[k] + bz[k + 1];
      std::swap(bz[k], bz[k + 1]);
      std::swap(bk[k], bk[k + 1]);
    }
    --end;
  }
  int r = 0;
  for (int b = 0; b < nb && bk[b]; ++b) r += bz[b];
  return r;
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

void schur_select(int n, std::vector<cplx>& T, std::vector<cplx>& Z, const std::vector<char>& keep) {
  // walk up from the bottom; every entry not kept sinks to the end of the kept block
  std::vector<char> kp(keep);
  int end = n;
  for (int i = n - 1; i >= 0; --i) {
    if (kp[i]) continue;
    for (int k = i; k < end - 1; ++k) {
      swap_adjacent(n, T, Z, k);
      std::swap(kp[k], kp[k + 1]);
    }
    --end;
  }
}

namespace {

// A real 2x2 block B = [[a, b], [c, d]] triangularised by the unitary
// G = [[v1, -conj(v2)], [v2, conj(v1)]] whose first column is a unit
// eigenvector of B (the rotation schur_complexify applies):
// G^H B G = [[m1, beta], [0, m2]].
struct Block2 {
  cplx v1, v2, m1, m2, beta;
  bool pair;   // complex-conjugate eigenvalues: m2 is taken as conj(m1)
};

Block2 block2(double a, double b, double c, double d) {
  const cplx half = 0.5 * (a - d);
  const cplx disc = std::sqrt(half * half + b * c);
  const cplx lam = 0.5 * (a + d) + disc;
  cplx v1 = b, v2 = lam - a;
  if (std::abs(v1) + std::abs(v2) < std::abs(lam - d) + std::abs(c)) { v1 = lam - d; v2 = c; }
  const double nv = std::sqrt(std::norm(v1) + std::norm(v2));
  v1 /= nv;
  v2 /= nv;
  const cplx g00 = a * v1 + b * v2, g10 = c * v1 + d * v2;   // B times the first column of G
  const cplx g01 = -a * std::conj(v2) + b * std::conj(v1);    // B times the second column
  const cplx g11 = -c * std::conj(v2) + d * std::conj(v1);
  Block2 r;
  r.v1 = v1;
  r.v2 = v2;
  r.m1 = std::conj(v1) * g00 + std::conj(v2) * g10;
  r.beta = std::conj(v1) * g01 + std::conj(v2) * g11;
  r.pair = (half * half + b * c).real() < 0.0;
  r.m2 = r.pair ? std::conj(r.m1) : -v2 * g01 + v1 * g11;
  return r;
}

inline bool block_starts2(int n, const std::vector<double>& T, int i) {
  return i + 1 < n && T[(i + 1) + (size_t)i * n] != 0.0;
}

}  // namespace

void schur_real_eigvals(int n, const std::vector<double>& T, std::vector<cplx>& theta) {
  theta.assign(n, cplx(0.0));
  for (int i = 0; i < n;) {
    if (block_starts2(n, T, i)) {
      const Block2 g = block2(T[i + (size_t)i * n], T[i + (size_t)(i + 1) * n], T[(i + 1) + (size_t)i * n],
                              T[(i + 1) + (size_t)(i + 1) * n]);
      theta[i] = g.m1;
      theta[i + 1] = g.m2;
      i += 2;
    } else {
      theta[i] = T[i + (size_t)i * n];
      i += 1;
    }
  }
}

void schur_eigvecs_real(int n, const std::vector<double>& T, const std::vector<double>& Q,
                        const std::vector<cplx>& theta, std::vector<cplx>& Y, double cluster_tol,
                        const std::vector<int>* which, bool schur_basis) {
  auto t = [&](int i, int j) { return T[i + (size_t)j * n]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(theta[i]));
  if (scale == 0.0) scale = 1.0;
  const double ctol = cluster_tol * scale;
  const double tiny = std::numeric_limits<double>::min() / std::numeric_limits<double>::epsilon();
  auto solve1 = [&](cplx rhs, cplx d) -> cplx {   // x with d x = rhs, clustered diagonal -> 0
    if (std::abs(d) <= ctol) return 0.0;
    if (std::abs(d) < tiny) d = tiny;
    return rhs / d;
  };
  // block of every position: its first row and size
  std::vector<int> bstart(n), bsize(n);
  for (int i = 0; i < n;) {
    const int sz = block_starts2(n, T, i) ? 2 : 1;
    for (int u = 0; u < sz; ++u) { bstart[i + u] = i; bsize[i + u] = sz; }
    i += sz;
  }
  Y.assign((size_t)n * n, cplx(0.0));
  std::vector<char> done(n, 0);
  std::vector<cplx> x(n);
  std::vector<double> yr(n), yi(n);
  const int nk = which ? (int)which->size() : n;
  for (int kk = 0; kk < nk; ++kk) {
    const int k = which ? (*which)[kk] : kk;
    if (done[k]) continue;
    const cplx lam = theta[k];
    const int kb = bstart[k], kend = kb + bsize[k] - 1;
    std::fill(x.begin(), x.begin() + kend + 1, cplx(0.0));
    // the eigenvector on its own block (triangularised coordinates w, x = G w)
    if (bsize[k] == 1) {
      x[k] = 1.0;
    } else {
      const Block2 g = block2(t(kb, kb), t(kb, kb + 1), t(kb + 1, kb), t(kb + 1, kb + 1));
      cplx w0 = 1.0, w1 = 0.0;
      if (k == kb + 1) {
        w1 = 1.0;
        w0 = solve1(-g.beta, g.m1 - lam);
      }
      x[kb] = g.v1 * w0 - std::conj(g.v2) * w1;
      x[kb + 1] = g.v2 * w0 + std::conj(g.v1) * w1;
    }
    // back-substitution through the blocks above, bottom to top
    for (int i = kb - 1; i >= 0;) {
      const int i0 = bstart[i];
      if (bsize[i] == 1) {
        cplx s = 0.0;
        for (int j = i + 1; j <= kend; ++j) s += t(i, j) * x[j];
        x[i] = solve1(-s, t(i, i) - lam);
      } else {
        cplx s0 = 0.0, s1 = 0.0;
        for (int j = i0 + 2; j <= kend; ++j) {
          s0 += t(i0, j) * x[j];
          s1 += t(i0 + 1, j) * x[j];
        }
        const Block2 g = block2(t(i0, i0), t(i0, i0 + 1), t(i0 + 1, i0), t(i0 + 1, i0 + 1));
        const cplx r0 = std::conj(g.v1) * s0 + std::conj(g.v2) * s1, r1 = -g.v2 * s0 + g.v1 * s1;
        const cplx w1 = solve1(-r1, g.m2 - lam);
        const cplx w0 = solve1(-r0 - g.beta * w1, g.m1 - lam);
        x[i0] = g.v1 * w0 - std::conj(g.v2) * w1;
        x[i0 + 1] = g.v2 * w0 + std::conj(g.v1) * w1;
      }
      i = i0 - 1;
    }
    // y = Q x (or x itself in the Schur basis), unit 2-norm
    std::fill(yr.begin(), yr.end(), 0.0);
    std::fill(yi.begin(), yi.end(), 0.0);
    if (schur_basis) {
      for (int j = 0; j <= kend; ++j) {
        yr[j] = x[j].real();
        yi[j] = x[j].imag();
      }
    } else {
      for (int j = 0; j <= kend; ++j) {
        const double xr = x[j].real(), xi = x[j].imag();
        const double* q = &Q[(size_t)j * n];
        for (int i = 0; i < n; ++i) {
          yr[i] += q[i] * xr;
          yi[i] += q[i] * xi;
        }
      }
    }
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm += yr[i] * yr[i] + yi[i] * yi[i];
    nrm = std::sqrt(nrm);
    cplx* y = &Y[(size_t)k * n];
    for (int i = 0; i < n; ++i) y[i] = cplx(yr[i] / nrm, yi[i] / nrm);
    done[k] = 1;
    // the conjugate eigenvalue of a complex pair: the conjugate vector
    if (bsize[k] == 2 && k == kb &&
        block2(t(kb, kb), t(kb, kb + 1), t(kb + 1, kb), t(kb + 1, kb + 1)).pair) {
      cplx* y2 = &Y[(size_t)(kb + 1) * n];
      for (int i = 0; i < n; ++i) y2[i] = std::conj(y[i]);
      done[kb + 1] = 1;
    }
  }
}

void schur_eigvecs(int n, const std::vector<cplx>& T, const std::vector<cplx>& Z,
                   std::vector<cplx>& Y, double cluster_tol, const std::vector<int>* which) {
  auto t = [&](int i, int j) { return T[i + (size_t)j * n]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(t(i, i)));
  if (scale == 0.0) scale = 1.0;
  const double tiny = std::numeric_limits<double>::min() / std::numeric_limits<double>::epsilon();
  Y.assign((size_t)n * n, cplx(0.0));
  std::vector<cplx> x(n);
  const int nk = which ? (int)which->size() : n;
  for (int kk = 0; kk < nk; ++kk) {
    const int k = which ? (*which)[kk] : kk;
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

int sym_eig_jacobi(int n, const double* Ain, std::vector<double>& w, std::vector<double>& Z) {
  std::vector<double> A((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) A[i + (size_t)j * n] = A[j + (size_t)i * n] = Ain[i + (size_t)j * n];
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[i + (size_t)i * n] = 1.0;
  double fro = 0.0;
  for (double x : A) fro += x * x;
  const double eps = std::numeric_limits<double>::epsilon();
  const double floor_abs = eps * eps * std::sqrt(fro);
  // a pair is rotated only while |a_pq| exceeds eps sqrt(|a_pp a_qq|) (below
  // that it no longer moves the diagonal in working precision); a sweep with
  // no rotation ends the iteration
  int sweeps = 0;
  bool rotated = true;
  for (; sweeps < 50 && rotated; ++sweeps) {
    rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p + (size_t)q * n];
        const double app = A[p + (size_t)p * n], aqq = A[q + (size_t)q * n];
        if (std::abs(apq) <= std::max(eps * std::sqrt(std::abs(app * aqq)), floor_abs)) continue;
        rotated = true;
        // rotation [c s; -s c] with tan = t the smaller root of t^2 + 2 tau t - 1 = 0
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // A <- J^T A J on rows / columns p and q
        for (int k = 0; k < n; ++k) {
          const double akp = A[k + (size_t)p * n], akq = A[k + (size_t)q * n];
          A[k + (size_t)p * n] = c * akp - s * akq;
          A[k + (size_t)q * n] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p + (size_t)k * n], aqk = A[q + (size_t)k * n];
          A[p + (size_t)k * n] = c * apk - s * aqk;
          A[q + (size_t)k * n] = s * apk + c * aqk;
        }
        A[p + (size_t)q * n] = A[q + (size_t)p * n] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double zkp = Z[k + (size_t)p * n], zkq = Z[k + (size_t)q * n];
          Z[k + (size_t)p * n] = c * zkp - s * zkq;
          Z[k + (size_t)q * n] = s * zkp + c * zkq;
        }
      }
  }
  if (rotated) return -1;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int a, int b) { return A[a + (size_t)a * n] < A[b + (size_t)b * n]; });
  w.resize(n);
  std::vector<double> Zs((size_t)n * n);
  for (int i = 0; i < n; ++i) {
    w[i] = A[idx[i] + (size_t)idx[i] * n];
    for (int k = 0; k < n; ++k) Zs[k + (size_t)i * n] = Z[k + (size_t)idx[i] * n];
  }
  Z.swap(Zs);
  return sweeps;
}

}  // namespace riga
