// A complex target shift sigma = a + ib on the real QEP (Sec. 4.1.1 with a
// complex shift; Alg. 2's target inside the complex spectrum region).
//
// The Krylov iteration runs on the real part of the shift-and-invert operator
// (Parlett and Saad, 1987), Re S(sigma) v = Re((A - sigma B)^{-1} B v), whose
// eigenvectors are the pencil's.  One application needs x = -Q(sigma)^{-1} t
// with the complex Q(sigma) = R + iJ,
//   R = (a^2 - b^2) M + a C + K,   J = b (2a M + C),
// solved in the real form of -i Q(sigma) = J - iR on two unknowns per dof
// (2d: Re x_d, 2d + 1: Im x_d):
//   [[J, R], [-R, J]] = J (x) I + R (x) E,  E = [[0, 1], [-1, 0]],
// whose symmetric part J (x) I is positive definite when J is (b > 0 and
// 2a M + C positive definite), so Gaussian elimination without pivoting runs
// on it with positive pivots (the LU fronts of the gyroscopic damping).
#include "kernels.hpp"

namespace riga {

namespace {

constexpr int CS_THREADS = 256;

// One wave per base row i: the entries q of row i fill row 2i (J, R) and row
// 2i + 1 (-R, J) of the doubled pattern, entry 2 (q - rowptr_i) + d; the
// symmetric part goes to Kr, the skew part to Cr and its transpose -Cr to Ctr.
__global__ __launch_bounds__(CS_THREADS) void k_realform_values(
    int64_t n, const int64_t* __restrict__ rowptr, const double* __restrict__ K, const double* __restrict__ M,
    const double* __restrict__ C, double a, double b, double* __restrict__ Kr, double* __restrict__ Cr,
    double* __restrict__ Ctr) {
  const int64_t i = ((int64_t)blockIdx.x * CS_THREADS + threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  if (i >= n) return;
  const int64_t r0 = rowptr[i];
  const int len = (int)(rowptr[i + 1] - r0);
  const int64_t o0 = 4 * r0, o1 = 4 * r0 + 2 * (int64_t)len;
  const double cm = a * a - b * b, cj = 2.0 * a * b;
  for (int q = lane; q < len; q += 64) {
    const double m = M[r0 + q], c = C[r0 + q], k = K[r0 + q];
    const double J = cj * m + b * c;
    const double R = cm * m + a * c + k;
    const int64_t e0 = o0 + 2 * q, e1 = o1 + 2 * q;
    *reinterpret_cast<double2*>(Kr + e0) = make_double2(J, 0.0);
    *reinterpret_cast<double2*>(Kr + e1) = make_double2(0.0, J);
    *reinterpret_cast<double2*>(Cr + e0) = make_double2(0.0, R);
    *reinterpret_cast<double2*>(Cr + e1) = make_double2(-R, 0.0);
    *reinterpret_cast<double2*>(Ctr + e0) = make_double2(0.0, -R);
    *reinterpret_cast<double2*>(Ctr + e1) = make_double2(R, 0.0);
  }
}

// Right-hand side of the real form for x = -Q^{-1} t, t = (a M + C) v_u + M v_l
// + i b M v_u:  -i (-t) = -Im t + i Re t, i.e. (2d, 2d + 1) = (-b MX_d,
// a MX_d + CW_d), with MX = M v_u and CW = C v_u + M v_l.
__global__ __launch_bounds__(CS_THREADS) void k_cshift_rhs(int64_t n, int nb, const double* __restrict__ MX,
                                                           const double* __restrict__ CW, int64_t ld, double a,
                                                           double b, double* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * CS_THREADS + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t col = t / n, d = t - col * n;
  const double mx = MX[d + col * ld], cw = CW[d + col * ld];
  *reinterpret_cast<double2*>(out + col * ldo + 2 * d) = make_double2(-b * mx, a * mx + cw);
}

// The operator's output from x (complex, interleaved): r_u = Re x,
// r_l = Re(sigma x + v_u) = a Re x - b Im x + v_u.
__global__ __launch_bounds__(CS_THREADS) void k_cshift_out(int64_t n, int nb, const double* __restrict__ x,
                                                           int64_t ldx, double a, double b,
                                                           const double* __restrict__ vu, int64_t ldv,
                                                           double* __restrict__ ru, double* __restrict__ rl,
                                                           int64_t ldr) {
  const int64_t t = (int64_t)blockIdx.x * CS_THREADS + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t col = t / n, d = t - col * n;
  const double2 v = *reinterpret_cast<const double2*>(x + col * ldx + 2 * d);
  ru[d + col * ldr] = v.x;
  rl[d + col * ldr] = a * v.x - b * v.y + vu[d + col * ldv];
}

// -i b for complex b (interleaved): (Re, Im) -> (Im, -Re), the real form's
// right-hand side of Q x = b.
__global__ __launch_bounds__(CS_THREADS) void k_times_minus_i(int64_t m, const double* __restrict__ in,
                                                              double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * CS_THREADS + threadIdx.x;
  if (t >= m) return;
  const double2 v = *reinterpret_cast<const double2*>(in + 2 * t);
  *reinterpret_cast<double2*>(out + 2 * t) = make_double2(v.y, -v.x);
}

unsigned grid_of(int64_t work) { return (unsigned)((work + CS_THREADS - 1) / CS_THREADS); }

}  // namespace

void launch_realform_values(int64_t n, const int64_t* rowptr, const double* K, const double* M, const double* C,
                            double a, double b, double* Kr, double* Cr, double* Ctr, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_realform_values, dim3(grid_of(n * 64)), dim3(CS_THREADS), 0, st, n, rowptr, K, M, C, a, b,
                     Kr, Cr, Ctr);
}

void launch_cshift_rhs(int64_t n, int nb, const double* MX, const double* CW, int64_t ld, double a, double b,
                       double* out, int64_t ldo, hipStream_t st) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_cshift_rhs, dim3(grid_of(n * nb)), dim3(CS_THREADS), 0, st, n, nb, MX, CW, ld, a, b, out,
                     ldo);
}

void launch_cshift_out(int64_t n, int nb, const double* x, int64_t ldx, double a, double b, const double* vu,
                       int64_t ldv, double* ru, double* rl, int64_t ldr, hipStream_t st) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_cshift_out, dim3(grid_of(n * nb)), dim3(CS_THREADS), 0, st, n, nb, x, ldx, a, b, vu, ldv, ru,
                     rl, ldr);
}

void launch_times_minus_i(int64_t m, const double* in, double* out, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_times_minus_i, dim3(grid_of(m)), dim3(CS_THREADS), 0, st, m, in, out);
}

}  // namespace riga
