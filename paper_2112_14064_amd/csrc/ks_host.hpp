// Host part of one Krylov--Schur cycle on the projected matrix (Alg. 2 with
// the restart of Sec. 4.1.3), and the per-pair arithmetic of the eigenpair
// post-processing.  Shared by the single-problem and the batched drivers.
#pragma once
#include <complex>
#include <vector>

#include "small_eig.hpp"

namespace riga {

struct KsCycle {
  std::vector<double> TR, QR;      // real Schur form of H_k and its vectors (k x k)
  std::vector<cplx> T, Z, Y;       // complex Schur form and its vectors (formed by the restart
                                   // only when the real reordering fails), Ritz vectors (k x k,
                                   // formed by ks_ritz_vectors)
  std::vector<cplx> X;             // the wanted Ritz vectors in the Schur basis (k x k)
  int k = 0;                       // dimension of the last Rayleigh--Ritz
  std::vector<cplx> theta;         // Ritz values of S
  std::vector<int> ord;            // positions by |theta| descending, clusters kept together
  int nw = 0;                      // wanted values: nev extended to the end of its cluster
  int nconv = 0;                   // wanted values whose Ritz residual passes the test
  std::vector<int> wanted;         // ord[0 .. nw)
  std::vector<char> conv;          // per position of TR: a wanted value that passed the test
  double tol = 0.0;                // the test's tolerance (kept for the restart's locking)
  int nlock = 0;                   // leading columns the last restart decoupled (locked)
  int r = 0;                       // kept dimension after the restart
  std::vector<double> Qe;          // (k+b) x (r+b) combination of the basis, column-major
  std::vector<double> Hn;          // projected matrix after the restart, ldh x ldh
  bool real_restart = false;       // the last restart reordered the real Schur form
};

// Rayleigh--Ritz on H_k (eq. ArnoldiRitz): H is ldh x ldh column-major with H_k
// in rows/columns 0..k and the residual rows E in rows k..k+b.  A Ritz pair
// counts as converged when ||E y|| <= tol |theta|.  Returns -1 if the Schur
// iteration failed.
int ks_ritz(const std::vector<double>& H, int ldh, int k, int b, int nev, double tol, KsCycle& c);

// Ritz vectors Y = Q X of the wanted values of the last ks_ritz (only the
// final cycle needs them; the convergence test works in the Schur basis).
void ks_ritz_vectors(KsCycle& c);

// Krylov--Schur restart after ks_ritz: keep the `keep` Ritz values nearest the
// shift (0: nev + (k - nev)/2; never fewer than nev; extended to whole
// clusters), real Schur basis of their span, the new projected matrix
// [T; E Q] and the combination Qe = [Q 0; 0 I].  Converged values are moved
// to the front of the kept ones; a leading run of them whose Schur vectors
// couple to the residual block by at most tol |theta| is locked: that part of
// E Q is set to zero, so the next projected matrix is block upper triangular
// and its Schur form only iterates on the trailing block.
void ks_restart(const std::vector<double>& H, int ldh, int k, int b, int m, int nev, int keep, KsCycle& c);

// Forms of a complex vector u = a + i b given the 11 sums
// a^T M a, b^T M b, a^T M b, a^T C a, b^T C b, a^T C b, a^T K a, b^T K b, a^T K b, a^T a, b^T b.
struct PairForms {
  cplx qm, qc, qk;   // unconjugated u^T M u, u^T C u, u^T K u
  double uMu;        // u^H M u
  double unorm2;     // u^H u
};
PairForms pair_forms(const double f[11]);
// Root of u^T Q(lam) u = 0 nearest the Ritz value (two-sided Rayleigh
// functional of the complex-symmetric pencil), or the Ritz value if the roots
// are not finite.
cplx rayleigh_polish(const PairForms& pf, cplx ritz);
// eta = ||Q(lam) u|| / ((|lam|^2 ||M||_1 + |lam| ||C||_1 + ||K||_1) ||u||) from
// ||Q(lam) u||^2; norms = {||K||_1, ||C||_1, ||M||_1}.
double scaled_residual(double resid2, cplx lam, const double norms[3], double unorm2);

}  // namespace riga
