// Dense eigen-decomposition of the small projected matrix of the Krylov
// iteration (Rayleigh--Ritz, eq. ArnoldiRitz) and the Krylov--Schur restart
// helpers (Sec. 4.1.3).  Host code; sizes are the subspace dimension (<= ~100).
#pragma once
#include <complex>
#include <vector>

namespace riga {

using cplx = std::complex<double>;

// A = Z T Z^H for a real n x n column-major A: T upper triangular, Z unitary
// (both n x n column-major complex).  Householder reduction to Hessenberg
// form, then single-shift complex QR iterations with Wilkinson shifts.
// Returns 0, or -1 if the iteration did not converge.
int schur_complex(int n, const double* A, std::vector<cplx>& T, std::vector<cplx>& Z);

// The real Schur form A = Q T Q^T behind schur_complex: T quasi upper
// triangular (1x1 blocks and 2x2 blocks of complex-conjugate pairs, nonzero
// subdiagonal), Q orthogonal.  Returns 0, or -1 if the iteration failed.
int schur_real(int n, const double* A, std::vector<double>& T, std::vector<double>& Q);
// The complex Schur form of a real one (each 2x2 block triangularised):
// diagonal position i of the complex T is position i of the real T.
void schur_complexify(int n, const std::vector<double>& TR, const std::vector<double>& QR, std::vector<cplx>& T,
                      std::vector<cplx>& Z);
// Reorder a real Schur form so that the blocks at positions with keep[i] != 0
// come first, their relative order kept, by exchanges of adjacent blocks in
// real arithmetic.  Returns the kept dimension r (the leading r columns of Q
// span the kept invariant subspace and T[0:r, 0:r] is its quasi-triangular
// form), or -1 when an exchange is ill conditioned or the mask splits a 2x2
// block; T and Q are then unusable.
int schur_select_real(int n, std::vector<double>& T, std::vector<double>& Q, const std::vector<char>& keep);

// Reorder the Schur form so that the eigenvalues at positions order[0..k-1]
// (positions in the current T) come first, in that order.
void schur_reorder(int n, std::vector<cplx>& T, std::vector<cplx>& Z, const std::vector<int>& order);

// Eigenvectors of A from its Schur form, columns of Y (n x n) normalised to unit
// 2-norm.  Diagonal entries of T that agree to `cluster_tol` (relative to the
// largest |T_ii|) are treated as one multiple eigenvalue whose eigenvectors
// are taken from the Schur basis (the coupling of a semisimple multiple
// eigenvalue vanishes in exact arithmetic).
// Only the columns listed in `which` are computed when it is not null (the
// others are left zero).
void schur_eigvecs(int n, const std::vector<cplx>& T, const std::vector<cplx>& Z,
                   std::vector<cplx>& Y, double cluster_tol, const std::vector<int>* which = nullptr);

// Eigenvalues of a real Schur form T in the order of its diagonal: a 2x2
// block gives the diagonal of its triangularised form (the values at the same
// positions of schur_complexify's T).
void schur_real_eigvals(int n, const std::vector<double>& T, std::vector<cplx>& theta);
// The eigenvectors of schur_eigvecs computed from the real Schur form
// A = Q T Q^T (theta from schur_real_eigvals): back-substitution through the
// quasi-triangular T with each 2x2 block triangularised on the fly, so the
// same clustering rule applies per diagonal position; the vector of the
// second eigenvalue of a complex-conjugate block is the conjugate of the first.
// With schur_basis, Y holds the vectors in the coordinates of the Schur basis
// (the eigenvectors of T, unit 2-norm); Q times them gives the eigenvectors
// of A.
void schur_eigvecs_real(int n, const std::vector<double>& T, const std::vector<double>& Q,
                        const std::vector<cplx>& theta, std::vector<cplx>& Y, double cluster_tol,
                        const std::vector<int>* which = nullptr, bool schur_basis = false);

// Reorder the Schur form so that the diagonal entries with keep[i] != 0 come
// first (their relative order kept) with the fewest adjacent exchanges: each
// entry not kept moves down past the kept ones below it.
void schur_select(int n, std::vector<cplx>& T, std::vector<cplx>& Z, const std::vector<char>& keep);

// Eigenvalues w (ascending) and orthonormal eigenvectors Z (n x n,
// column-major, column i for w[i]) of a real symmetric n x n column-major A
// (only its lower triangle is read) by the cyclic Jacobi method: plane
// rotations that annihilate one off-diagonal pair at a time, swept row by row
// until no pair exceeds eps sqrt(|a_pp a_qq|) (Golub and Van Loan, Sec. 8.5).
// Returns the number of sweeps, or -1 without convergence in 50 sweeps.
int sym_eig_jacobi(int n, const double* A, std::vector<double>& w, std::vector<double>& Z);

// Real orthonormal basis Q (n x r, column-major) of span{Re z, Im z} over the
// first k columns of Z (n x n).  When those columns span a subspace closed
// under conjugation, r == k.  Returns r.
int realify(int n, int k, const std::vector<cplx>& Z, std::vector<double>& Q);

}  // namespace riga
