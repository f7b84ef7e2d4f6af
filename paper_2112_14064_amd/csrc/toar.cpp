// Block Krylov--Schur on the shift-and-invert operator of the companion
// pencil (Alg. 2, eq. BlockOperatorVector) with the Krylov basis in compact
// two-level (TOAR) form
//   V_j = [U Q1; U Q2],   U: N x r, U^T U = I,   Q = [Q1; Q2]: 2r x j, Q^T Q = I,
// so that V_j^T V_j = I and the N-long storage is U alone (r = j + b columns
// instead of the 2N x j of V; the SOAR-type methods cited in Sec. 4.2.1).
// It holds because r_l = sigma r_u + v_u in eq. BlockOperatorVector: the
// lower block of the operator's image lies in span(U) once the upper block
// r_u is added to U.  The inner product is the Euclidean one of the 2N-space
// (TOAR's); the eigenvalues the iteration converges to are those of the
// full-basis iteration, whose B-inner product is a choice of the paper's
// Alg. 2 that a compact basis would have to carry as U^T M U.
//
// Block step at processed columns k (basis V_{k+b}, r = k + 2b columns of U):
//   [v_u | v_l] = U P                          (P: coordinates of block k)
//   r_u = -Q^{-1}((sigma M + C) v_u + M v_l)   (sweeps; M v_l by sum factorisation)
//   r_u = U s + u_new T                        (CGS2 against U, Euclidean; U += u_new)
//   x_u = [s; T],  x_l = sigma x_u + [q1; 0]   (coordinates of the image)
//   x -> CGS2 against Q, normalised: H's column block and Q's new columns.
// Restart (Krylov--Schur, host): Q <- Q Qe, then U is compressed to the
// range of [Q1 Q2] (Householder QR with column pivoting), r = kept + 2b.
#include "problem.hpp"
#include "ks_host.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

using riga::cplx;

namespace riga {
namespace detail {

namespace {

void ensure_toar(riga_problem* h, int cols, int b) {
  if (h->tw_cols >= cols && h->tw_b >= b) return;
  h->clear_graphs();
  for (double* p : {h->tU, h->tU2, h->tX, h->tW, h->tRu, h->tRl, h->tTv, h->tQ, h->tS, h->tP, h->tsmall, h->tH})
    h->dfree(p);
  h->dfree(h->tflag);
  cols = std::max<int>(cols, (int)h->tw_cols);
  b = std::max<int>(b, (int)h->tw_b);
  const int64_t N = h->N();
  h->tU = h->dalloc<double>(N * cols);
  h->tU2 = h->dalloc<double>(N * cols);
  h->tX = h->dalloc<double>(N * 2 * b);
  h->tW = h->dalloc<double>(N * b);
  h->tRu = h->dalloc<double>(N * b);
  h->tRl = h->dalloc<double>(N * b);
  h->tTv = h->dalloc<double>(N * b);
  h->tQ = h->dalloc<double>((size_t)2 * cols * cols);
  h->tS = h->dalloc<double>((size_t)cols * 4);
  h->tP = h->dalloc<double>((size_t)cols * 8);
  h->tsmall = h->dalloc<double>((size_t)4 * cols * cols + 64);
  h->tH = h->dalloc<double>((size_t)cols * cols);
  h->tflag = h->dalloc<int>(4);
  h->tw_cols = cols;
  h->tw_b = b;
}

// Orthonormal W (r x rp, column-major) whose range holds the columns of A
// (r x nc, column-major) up to rounding: Householder QR with column pivoting
// (largest remaining norm first), W = the first rp columns of the orthogonal
// factor.  Returns the largest norm left in a column after rp steps relative
// to the largest column norm of A (zero in exact arithmetic when
// rank(A) <= rp).
// sum_i a[i] b[i] over [from, to) in four interleaved partial sums (a fixed
// order the compiler can keep in vector registers)
inline double dot4(const double* a, const double* b, int from, int to) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = from;
  for (; i + 3 < to; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < to; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

double range_basis(int r, int nc, std::vector<double> A, int rp, std::vector<double>& W) {
  std::vector<double> norm2(nc), v((size_t)rp * r, 0.0), beta(rp, 0.0);
  auto colnorm2 = [&](int c, int from) {
    const double* a = &A[(size_t)c * r];
    return dot4(a, a, from, r);
  };
  double amax = 0.0;
  for (int c = 0; c < nc; ++c) amax = std::max(amax, colnorm2(c, 0));
  amax = std::sqrt(amax);
  const int steps = std::min(rp, std::min(r, nc));
  for (int j = 0; j < steps; ++j) {
    int best = j;
    double bn = -1.0;
    for (int c = j; c < nc; ++c) {
      norm2[c] = colnorm2(c, j);   // recomputed: the sizes are small
      if (norm2[c] > bn) { bn = norm2[c]; best = c; }
    }
    if (best != j)
      for (int i = 0; i < r; ++i) std::swap(A[i + (size_t)j * r], A[i + (size_t)best * r]);
    // reflector H_j = I - beta v v^T with v[j] = 1, mapping A[j:, j] to -sign * alpha e_j
    const double x0 = A[j + (size_t)j * r];
    const double alpha = std::sqrt(bn);
    double* vj = &v[(size_t)j * r];
    if (alpha == 0.0) {
      beta[j] = 0.0;
      continue;
    }
    const double d = x0 >= 0.0 ? x0 + alpha : x0 - alpha;
    vj[j] = 1.0;
    for (int i = j + 1; i < r; ++i) vj[i] = A[i + (size_t)j * r] / d;
    double vv = 1.0;
    for (int i = j + 1; i < r; ++i) vv += vj[i] * vj[i];
    beta[j] = 2.0 / vv;
    for (int c = j; c < nc; ++c) {
      double* a = &A[(size_t)c * r];
      const double s = beta[j] * dot4(vj, a, j, r);
      for (int i = j; i < r; ++i) a[i] -= s * vj[i];
    }
  }
  double rest = 0.0;
  for (int c = steps; c < nc; ++c) rest = std::max(rest, colnorm2(c, steps));
  // W = H_0 H_1 ... H_{steps-1} I[:, 0:rp]
  W.assign((size_t)r * rp, 0.0);
  for (int c = 0; c < rp; ++c) W[c + (size_t)c * r] = 1.0;
  for (int j = steps - 1; j >= 0; --j) {
    if (beta[j] == 0.0) continue;
    const double* vj = &v[(size_t)j * r];
    for (int c = 0; c < rp; ++c) {
      double* w = &W[(size_t)c * r];
      const double s = beta[j] * dot4(vj, w, j, r);
      for (int i = j; i < r; ++i) w[i] -= s * vj[i];
    }
  }
  return amax > 0.0 ? std::sqrt(rest) / amax : 0.0;
}

// Cholesky G = R^T R of a small SPD matrix (n x n, column-major); false when
// a pivot falls below rel times its diagonal entry.
bool chol_upper(int n, const std::vector<double>& G, std::vector<double>& R, double rel) {
  R.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = 0.5 * (G[i + (size_t)j * n] + G[j + (size_t)i * n]);
      for (int t = 0; t < i; ++t) s -= R[t + (size_t)i * n] * R[t + (size_t)j * n];
      if (i == j) {
        if (!(s > rel * G[j + (size_t)j * n]) || !std::isfinite(s)) return false;
        R[j + (size_t)j * n] = std::sqrt(s);
      } else {
        R[i + (size_t)j * n] = s / R[i + (size_t)i * n];
      }
    }
  }
  return true;
}

}  // namespace

riga_status eigs_toar(riga_problem* h, const riga_options* opt, int nev, int b, int m, int maxit, double tol,
                      double* lam, double* X, double* eta, int* nconv, bool* fallback) {
  *fallback = false;
  const int64_t N = h->N();
  const int ldh = m + 2 * b;
  // U's column count reaches m + 2b: the tall products take at most 254 inner
  // columns and the compact kernel's tables hold 264 rows
  if (ldh > 254 || b > 4 || 2 * b > N) { *fallback = true; return RIGA_OK; }
  ensure_toar(h, ldh, b);
  hipStream_t st = h->st;
  double* U = h->tU;
  double* U2 = h->tU2;
  double* Q1 = h->tQ;
  double* Q2 = h->tQ + (size_t)ldh * ldh;
  double* h1 = h->tsmall;
  double* h2 = h->tsmall + (size_t)ldh * b;
  double* rbuf = h->tsmall + (size_t)2 * ldh * b;       // b x b
  double* dstage = h->tsmall + (size_t)2 * ldh * b + 16; // uploads of small matrices
  ck(hipEventRecord(h->ev0, st));
  ck(hipMemsetAsync(h->tflag, 0, sizeof(int), st));
  ck(hipMemsetAsync(h->tH, 0, sizeof(double) * (size_t)ldh * ldh, st));
  ck(hipMemsetAsync(h->tQ, 0, sizeof(double) * (size_t)2 * ldh * ldh, st));

  // --- start: U[:, 0:2b] an orthonormal basis of [x_u, x_l] (CholQR twice),
  // the start block's compact coordinates from U^T [x_u, x_l] -----------------
  const int b2 = 2 * b;
  if (opt->v0) {
    for (int q = 0; q < b; ++q) {
      ck(hipMemcpyAsync(h->tX + (size_t)q * N, opt->v0 + (size_t)q * 2 * N, N * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
      ck(hipMemcpyAsync(h->tX + (size_t)(b + q) * N, opt->v0 + (size_t)q * 2 * N + N, N * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    }
  } else {
    launch_random_fill(h->tX, N, b, N, opt->seed * 2 + 1, st);
    launch_random_fill(h->tX + (size_t)b * N, N, b, N, opt->seed * 2 + 2, st);
  }
  // G = A^T B for N x b2 blocks (column groups of at most 4)
  auto gram = [&](const double* A, const double* B, std::vector<double>& G) {
    double* dG = h->tsmall;
    for (int q0 = 0; q0 < b2; q0 += 4) {
      const int nq = std::min(4, b2 - q0);
      launch_dots(N, b2, A, nullptr, N, nq, B + (size_t)q0 * N, nullptr, N, h->d_part, dG + (size_t)q0 * b2, st);
    }
    std::vector<double> o((size_t)b2 * b2);
    ck(hipMemcpyAsync(o.data(), dG, o.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    ck(hipStreamSynchronize(st));
    G.assign((size_t)b2 * b2, 0.0);
    for (int q0 = 0; q0 < b2; q0 += 4) {
      const int nq = std::min(4, b2 - q0);
      for (int c = 0; c < b2; ++c)
        for (int q = 0; q < nq; ++q) G[c + (size_t)(q0 + q) * b2] = o[(size_t)q0 * b2 + (size_t)c * nq + q];
    }
  };
  auto upload = [&](const std::vector<double>& v, double* dst) {
    double* pin = h->pinned(v.size() + 8);
    std::memcpy(pin, v.data(), v.size() * sizeof(double));
    ck(hipMemcpyAsync(dst, pin, v.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ck(hipStreamSynchronize(st));   // the pinned block is reused by the next upload
  };
  {
    std::vector<double> G, R;
    gram(h->tX, h->tX, G);
    if (!chol_upper(b2, G, R, 1e-20)) { *fallback = true; return RIGA_OK; }   // start block not of full rank
    upload(upper_inverse(b2, R), dstage);
    launch_gemm_tall(N, h->tX, N, b2, dstage, b2, U2, N, st);
    std::vector<double> G2, R2;
    gram(U2, U2, G2);
    if (!chol_upper(b2, G2, R2, 1e-20)) { *fallback = true; return RIGA_OK; }
    upload(upper_inverse(b2, R2), dstage);
    launch_gemm_tall(N, U2, N, b2, dstage, b2, U, N, st);
    // coordinates C = U^T [x_u, x_l] (b2 x b2)
    std::vector<double> C;
    gram(U, h->tX, C);
    // start block x = [C[:, 0:b]; C[:, b:2b]] (2 b2 x b), orthonormalised
    std::vector<double> x((size_t)2 * b2 * b);
    for (int q = 0; q < b; ++q)
      for (int i = 0; i < b2; ++i) {
        x[i + (size_t)q * 2 * b2] = C[i + (size_t)q * b2];
        x[b2 + i + (size_t)q * 2 * b2] = C[i + (size_t)(b + q) * b2];
      }
    std::vector<double> Gx((size_t)b * b), Rx;
    for (int a = 0; a < b; ++a)
      for (int q = 0; q < b; ++q) {
        double s = 0.0;
        for (int i = 0; i < 2 * b2; ++i) s += x[i + (size_t)a * 2 * b2] * x[i + (size_t)q * 2 * b2];
        Gx[a + (size_t)q * b] = s;
      }
    if (!chol_upper(b, Gx, Rx, 1e-20)) { *fallback = true; return RIGA_OK; }
    const std::vector<double> Ri = upper_inverse(b, Rx);
    std::vector<double> Qh((size_t)2 * ldh * ldh, 0.0), Ph((size_t)b2 * b2, 0.0);
    for (int q = 0; q < b; ++q)
      for (int i = 0; i < 2 * b2; ++i) {
        double s = 0.0;
        for (int a = 0; a <= q; ++a) s += x[i + (size_t)a * 2 * b2] * Ri[a + (size_t)q * b];
        if (i < b2) {
          Qh[i + (size_t)q * ldh] = s;
          Ph[i + (size_t)q * b2] = s;
        } else {
          Qh[(size_t)ldh * ldh + (i - b2) + (size_t)q * ldh] = s;
          Ph[(i - b2) + (size_t)(b + q) * b2] = s;
        }
      }
    upload(Qh, h->tQ);
    upload(Ph, h->tP);
  }

  // --- block steps ------------------------------------------------------------
  int k = 0, r = b2;        // processed columns, columns of U (r = k + 2b)
  bool pre = false;         // the operator was already applied to block k
  int64_t n_fb = 0, n_mv = 0, n_vv = 0;
  double vv_bytes = 0.0, rs_bytes = 0.0, rs_flops = 0.0, drop_max = 0.0;
  auto enqueue_apply = [&](int rr) {
    launch_gemm_tall(N, U, N, rr, h->tP, b2, h->tX, N, st);
    launch_tensor_mk(h->ds, h->d_M1, h->d_K1, b, 1.0, 0.0, h->tX + (size_t)b * N, N, h->tW, N, nullptr, 0, 0.0, st);
    apply_block(h, b, h->tX, h->tW, N, h->tRu, h->tRl, h->tTv);
  };
  auto enqueue_orth = [&](int kk, int rr) {
    launch_dots(N, rr, U, nullptr, N, b, h->tRu, nullptr, N, h->d_part, h1, st);
    if (launch_toar_update_dots(N, rr, b, h1, U, N, h->tRu, N, h->d_part, h2, st) < 0) {
      launch_cgs_update(N, rr, b, h1, U, h->tRu, nullptr, nullptr, nullptr, nullptr, N, N, nullptr, st);
      launch_dots(N, rr, U, nullptr, N, b, h->tRu, nullptr, N, h->d_part, h2, st);
    }
    const int gblk = launch_cgs_update(N, rr, b, h2, U, h->tRu, nullptr, nullptr, nullptr, nullptr, N, N, h->d_part,
                                       st);
    launch_normalize_gemm3(N, rr, b, h1, h2, nullptr, h->d_part, gblk, h->tS, ldh, 0, h->tflag, rbuf, h->tRu,
                           U + (size_t)rr * N, nullptr, nullptr, nullptr, nullptr, N, st);
    launch_toar_compact(rr, kk, b, h->sigma, h->tS, ldh, Q1, Q2, ldh, h->tH, ldh, h->tflag, h->tP, st);
  };
  const bool graphs = !(opt->flags & 1);
  auto step = [&]() {
    if (graphs) {
      auto key = std::make_tuple(k, b, (const double*)U, (pre ? 1 : 0) | 4, ldh);
      auto it = h->graphs.find(key);
      if (it == h->graphs.end()) {
        ck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        if (!pre) enqueue_apply(r);
        enqueue_orth(k, r);
        hipGraph_t g = nullptr;
        ck(hipStreamEndCapture(st, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        ck(e);
        it = h->graphs.emplace(key, ex).first;
      }
      ck(hipGraphLaunch(it->second, st));
    } else {
      if (!pre) enqueue_apply(r);
      enqueue_orth(k, r);
    }
    pre = false;
    n_fb += b;
    n_mv += 3LL * b;
    n_vv += 5LL * r * b + 2LL * b * b;
    vv_bytes += 8.0 * (double)N * (4.0 * r + 6.0 * b);
    k += b;
    r += b;
  };

  KsCycle cyc;
  std::vector<double> H((size_t)ldh * ldh), Qh((size_t)2 * ldh * ldh);
  // pinned staging of a cycle: the downloads of H and Q (3 ldh^2), then the
  // restart's uploads W (ldh^2), Q (2 ldh^2), P (8 ldh) and H (ldh^2).  The
  // uploads are queued without waiting; the next cycle's download waits for
  // the stream, so no region is rewritten while a copy from it is in flight.
  const size_t L2 = (size_t)ldh * ldh;
  double* stage = h->pinned(7 * L2 + (size_t)8 * ldh + 64);
  double* up_W = stage + 3 * L2;
  double* up_Q = stage + 4 * L2;
  double* up_P = stage + 6 * L2;
  double* up_H = stage + 6 * L2 + (size_t)8 * ldh;
  int* dl_flag = (int*)(stage + 7 * L2 + (size_t)8 * ldh);
  int it = 0;
  bool converged = false, broke = false;
  double t_host = 0.0;
  for (;;) {
    while (k + b <= m) step();
    {
      ck(hipMemcpyAsync(stage, h->tH, sizeof(double) * L2, hipMemcpyDeviceToHost, st));
      ck(hipMemcpyAsync(stage + L2, h->tQ, sizeof(double) * 2 * L2, hipMemcpyDeviceToHost, st));
      ck(hipMemcpyAsync(dl_flag, h->tflag, sizeof(int), hipMemcpyDeviceToHost, st));
      ck(hipStreamSynchronize(st));
      std::memcpy(H.data(), stage, sizeof(double) * L2);
      std::memcpy(Qh.data(), stage + L2, sizeof(double) * 2 * L2);
      if (*dl_flag) { broke = true; break; }
    }
    // the first step of the next cycle applies the operator to block k, which
    // the restart keeps (as a vector): queue it now, on the current U and P
    enqueue_apply(r);
    pre = true;
    const auto th0 = std::chrono::steady_clock::now();
    if (ks_ritz(H, ldh, k, b, nev, tol, cyc) != 0) throw HipError{hipErrorUnknown};
    ++it;
    if (cyc.nconv == cyc.nw || it >= maxit) {
      t_host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
      converged = cyc.nconv == cyc.nw;
      break;
    }
    ks_restart(H, ldh, k, b, m, nev, opt->keep, cyc);
    const int kin = k + b, kout = cyc.r + b, rp = cyc.r + 2 * b;
    // Q <- Q Qe (r x kout each part), A = [Q1n Q2n]
    std::vector<double> A((size_t)r * 2 * kout, 0.0);
    for (int part = 0; part < 2; ++part) {
      const double* Qp = Qh.data() + (size_t)part * ldh * ldh;
      for (int c = 0; c < kout; ++c)
        for (int t = 0; t < kin; ++t) {
          const double e = cyc.Qe[t + (size_t)c * kin];
          if (e == 0.0) continue;
          for (int i = 0; i < r; ++i) A[i + (size_t)(part * kout + c) * r] += Qp[i + (size_t)t * ldh] * e;
        }
    }
    std::vector<double> W;
    drop_max = std::max(drop_max, range_basis(r, 2 * kout, A, rp, W));
    // compressed compact basis W^T [Q1n Q2n] and the packed block cyc.r
    std::memset(up_Q, 0, sizeof(double) * 2 * L2);
    for (int part = 0; part < 2; ++part)
      for (int c = 0; c < kout; ++c)
        for (int a = 0; a < rp; ++a) {
          const double s = dot4(&W[(size_t)a * r], &A[(size_t)(part * kout + c) * r], 0, r);
          up_Q[(size_t)part * L2 + a + (size_t)c * ldh] = s;
          if (c >= cyc.r) up_P[a + (size_t)(part * b + c - cyc.r) * rp] = s;
        }
    std::memcpy(up_W, W.data(), sizeof(double) * W.size());
    std::memcpy(up_H, cyc.Hn.data(), sizeof(double) * L2);
    ck(hipMemcpyAsync(dstage, up_W, sizeof(double) * W.size(), hipMemcpyHostToDevice, st));
    launch_gemm_tall(N, U, N, r, dstage, rp, U2, N, st);
    rs_bytes += 8.0 * (double)N * (r + rp);
    rs_flops += 2.0 * (double)N * r * rp;
    std::swap(U, U2);
    ck(hipMemcpyAsync(h->tQ, up_Q, sizeof(double) * 2 * L2, hipMemcpyHostToDevice, st));
    ck(hipMemcpyAsync(h->tP, up_P, sizeof(double) * (size_t)rp * b2, hipMemcpyHostToDevice, st));
    ck(hipMemcpyAsync(h->tH, up_H, sizeof(double) * L2, hipMemcpyHostToDevice, st));
    k = cyc.r;
    r = rp;
    t_host += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
  }
  // keep the current U in tU for the next call's buffers
  h->tU = U;
  h->tU2 = U2;
  if (broke) { *fallback = true; return RIGA_OK; }

  // --- eigenpairs: u = U (Q1 y) for the wanted Ritz vectors -----------------------
  ks_ritz_vectors(cyc);
  const int nw = (int)cyc.wanted.size();
  std::vector<double> Zr((size_t)r * nw, 0.0), Zi((size_t)r * nw, 0.0);
  for (int j = 0; j < nw; ++j)
    for (int c = 0; c < k; ++c) {
      const cplx y = cyc.Y[c + (size_t)cyc.wanted[j] * k];
      for (int i = 0; i < r; ++i) {
        const double q = Qh[i + (size_t)c * ldh];
        Zr[i + (size_t)j * r] += q * y.real();
        Zi[i + (size_t)j * r] += q * y.imag();
      }
    }
  ensure_post(h, nw);
  upload(Zr, dstage);
  launch_gemm_tall(N, U, N, r, dstage, nw, h->P, N, st);
  upload(Zi, dstage);   // (upload synchronises: the product above has read Zr)
  launch_gemm_tall(N, U, N, r, dstage, nw, h->P + (size_t)nw * N, N, st);
  const int conv_out = finish_pairs(h, cyc, nev, h->tsmall, lam, X, eta);
  ck(hipEventRecord(h->ev1, st));
  ck(hipStreamSynchronize(st));
  float ms = 0;
  ck(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  riga_stats_t& S = h->stats;
  S.t_eigs_ms = ms;
  S.n_it = it;
  S.n_fb = n_fb;
  S.t_host_ms = t_host;
  S.n_ir = h->mixed ? n_fb * h->ir_sweeps : 0;
  S.n_mv = n_mv + S.n_ir;
  S.n_vv = n_vv;
  {
    Plan& Pm = h->plan;
    Pm.ensure_symbolic();
    const double Nd = (double)N, nnz = (double)Pm.nnz, irs = h->mixed ? h->ir_sweeps : 0;
    const double vec = (double)n_fb, passes = vec / b * (1.0 + irs);
    S.bytes[RIGA_PHASE_FB] = passes * h->solve_bytes_now + vec * (1.0 + irs) * 16.0 * Nd;
    S.flops[RIGA_PHASE_FB] = vec * (1.0 + irs) * 4.0 * (double)Pm.sym_nnz_l;
    const double mv_bytes = 16.0 * Nd + (h->c_elem ? 8.0 * nnz + 16.0 * Nd : 16.0 * Nd);
    S.bytes[RIGA_PHASE_MV] = vec * (mv_bytes + 16.0 * Nd);
    S.flops[RIGA_PHASE_MV] = (double)n_mv * 2.0 * nnz;
    S.bytes[RIGA_PHASE_VV] = vv_bytes;
    S.flops[RIGA_PHASE_VV] = (double)n_vv * 2.0 * Nd;
    S.bytes[RIGA_PHASE_RESTART] = rs_bytes + 2.0 * 8.0 * Nd * (r + nw);
    S.flops[RIGA_PHASE_RESTART] = rs_flops + 2.0 * 2.0 * Nd * r * nw;
    S.bytes[RIGA_PHASE_IR] = irs > 0 ? vec / b * irs * 8.0 * nnz + vec * irs * 24.0 * Nd : 0.0;
    S.flops[RIGA_PHASE_IR] = vec * irs * 2.0 * nnz;
    const double pv = 2.0 * nw;
    S.bytes[RIGA_PHASE_POST] = std::ceil(pv / 8.0) * 24.0 * nnz + pv * 32.0 * Nd;
    S.flops[RIGA_PHASE_POST] = pv * 3.0 * 2.0 * nnz;
  }
  S.toar_drop = drop_max;
  if (nconv) *nconv = conv_out;
  return (converged && conv_out == nev) ? RIGA_OK : RIGA_WARN_NOT_CONVERGED;
}

}  // namespace detail
}  // namespace riga

extern "C" riga_status riga_selftest_range_basis(int r, int nc, const double* a, int rp, double* w,
                                                  double* drop) {
  if (r < 1 || nc < 1 || rp < 1 || rp > r || !a || !w || !drop) return RIGA_ERR_INVALID_ARG;
  return riga::detail::run([&]() -> riga_status {
    std::vector<double> A(a, a + (size_t)r * nc), W;
    *drop = riga::detail::range_basis(r, nc, A, rp, W);
    std::copy(W.begin(), W.end(), w);
    return RIGA_OK;
  });
}
