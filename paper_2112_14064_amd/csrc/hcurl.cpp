// 1-D matrices of the H(curl) space (Sec. 3.2, eq. HcurlBasis; Sec. 3.3, eq.
// DiscreteSpacesrIGA) on the host.  On the identity geometry every entry of
// the curl-curl and mass matrices of S^{p-1,p} x S^{p,p-1} is a product of
// 1-D integrals over the degree-(p-1) space A and the degree-p space B of one
// direction (the two directions use the same pair):
//   MA = int A_a A_a',  MB = int B_b B_b',  KB = int B_b' B_b'',  D = int A_a B_b'.
// They are integrated element by element with the (p+1)-point Gauss rule
// (exact: every integrand has degree at most 2p) from Cox--de Boor values
// (eq. BasisFunBi0 / BasisFunBip) and stored dense, row-major.
#include "problem.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace riga {
namespace detail {

namespace {

// Nonzero degree-q B-splines of knot vector t (element units) at u in span k
// (t[k] <= u < t[k+1]): N[r] is function k - q + r.
void basis_at(const std::vector<int>& t, int k, int q, double u, double* N) {
  double left[16], right[16];
  N[0] = 1.0;
  for (int j = 1; j <= q; ++j) {
    left[j] = u - (double)t[k + 1 - j];
    right[j] = (double)t[k + j] - u;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      const double tmp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

// Values V[r] and u-derivatives Dv[r] of the q+1 nonzero functions of a space
// at u in span k (functions k - q + r).
void values_derivs(const std::vector<int>& t, int k, int q, double u, double* V, double* Dv) {
  basis_at(t, k, q, u, V);
  double Nm[16];
  if (q > 0) basis_at(t, k, q - 1, u, Nm);
  for (int r = 0; r <= q; ++r) {
    const int i = k - q + r;
    double d = 0.0;
    if (q > 0) {
      const double d1 = (double)(t[i + q] - t[i]), d2 = (double)(t[i + q + 1] - t[i + 1]);
      if (r >= 1 && d1 > 0.0) d += Nm[r - 1] / d1;
      if (r <= q - 1 && d2 > 0.0) d -= Nm[r] / d2;
    }
    Dv[r] = (double)q * d;
  }
}

// Span of element e (knot indices in element units): the last k with t[k] <= e.
int span_of(const std::vector<int>& t, int e) {
  return (int)(std::upper_bound(t.begin(), t.end(), e) - t.begin()) - 1;
}

}  // namespace

void hcurl_1d(const Space1D& A, const Space1D& B, std::vector<double>& MA, std::vector<double>& MB,
              std::vector<double>& KB, std::vector<double>& D) {
  const int na = A.n, nb = B.n, ne = B.ne;
  MA.assign((size_t)na * na, 0.0);
  MB.assign((size_t)nb * nb, 0.0);
  KB.assign((size_t)nb * nb, 0.0);
  D.assign((size_t)na * nb, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre(B.p + 1, gx, gw);
  const double h = 1.0 / (double)ne;
  double VA[16], DA[16], VB[16], DB[16];
  for (int e = 0; e < ne; ++e) {
    const int ka = span_of(A.knots, e), kb = span_of(B.knots, e);
    for (size_t g = 0; g < gx.size(); ++g) {
      const double u = (double)e + 0.5 * (gx[g] + 1.0);
      const double w = 0.5 * gw[g];
      values_derivs(A.knots, ka, A.p, u, VA, DA);
      values_derivs(B.knots, kb, B.p, u, VB, DB);
      for (int r = 0; r <= A.p; ++r) {
        const int a = ka - A.p + r - A.off;
        if (a < 0 || a >= na) continue;
        for (int r2 = 0; r2 <= A.p; ++r2) {
          const int a2 = ka - A.p + r2 - A.off;
          if (a2 >= 0 && a2 < na) MA[(size_t)a * na + a2] += w * VA[r] * VA[r2] * h;
        }
        for (int s2 = 0; s2 <= B.p; ++s2) {
          const int b2 = kb - B.p + s2 - B.off;
          // d/dx = ne d/du and dx = h du: the factors cancel
          if (b2 >= 0 && b2 < nb) D[(size_t)a * nb + b2] += w * VA[r] * DB[s2];
        }
      }
      for (int s = 0; s <= B.p; ++s) {
        const int b = kb - B.p + s - B.off;
        if (b < 0 || b >= nb) continue;
        for (int s2 = 0; s2 <= B.p; ++s2) {
          const int b2 = kb - B.p + s2 - B.off;
          if (b2 < 0 || b2 >= nb) continue;
          MB[(size_t)b * nb + b2] += w * VB[s] * VB[s2] * h;
          KB[(size_t)b * nb + b2] += w * DB[s] * DB[s2] * (double)ne;
        }
      }
    }
  }
}

}  // namespace detail
}  // namespace riga
