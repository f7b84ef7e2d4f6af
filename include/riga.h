/*
 * riga.h -- C ABI of the MI355X shift-and-invert solver for the damped-wave
 * quadratic eigenvalue problem (K + lam C + lam^2 M) u = 0 discretised with
 * maximum-continuity IGA or refined IGA (rIGA) B-splines on the unit square.
 *
 * Paper: Hashemian, Garcia, Pardo, Calo, "Performance of refined isogeometric
 * analysis in solving quadratic eigenvalue problems" (arXiv 2112.14064).
 *
 * The calls follow the input/output statement of the paper's quadratic
 * eigen-procedure (Sec. 4.2.1, Alg. 2): system matrices K, C, M; a target
 * shift; the number of requested eigenpairs; the Krylov subspace size; an
 * initial vector; a tolerance -> eigenpairs.
 *
 * Conventions (all entry points):
 *   - Dofs are the tensor-product B-splines B_i(x) B_j(y) that vanish on the
 *     boundary (homogeneous Dirichlet: the first and last 1-D function of each
 *     direction are removed), numbered lexicographically, x fastest:
 *     dof = j * n1d + i.
 *   - "device" pointers are HIP device memory owned by the caller and must stay
 *     valid for the duration of the call; "host" pointers are ordinary memory.
 *     The library owns everything it allocates internally (matrices, factor,
 *     Krylov workspace) and frees it in riga_destroy.
 *   - All work is ordered after the caller's earlier work on the stream given
 *     to riga_create; riga_eigs runs its Krylov loop on a stream owned by the
 *     handle (fenced to the caller's stream with an event).  Calls return
 *     after the result they report is known: riga_factor, riga_eigs and
 *     riga_adjoint synchronise the stream; riga_assemble, riga_solve_q and
 *     riga_apply_op return as soon as the work is queued.
 *   - A negative status is an error: outputs are not written (except where a
 *     diagnostic such as *bad_pivot is documented).  A positive status is a
 *     warning: outputs are valid as documented.
 *   - A handle is not thread-safe: use one handle per host thread / stream.
 *   - Floating-point arguments and results are IEEE binary64.
 */
#ifndef RIGA_H
#define RIGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct riga_problem riga_problem;

typedef enum {
  RIGA_OK = 0,
  RIGA_ERR_INVALID_ARG = -1,   /* bad size, degree, pointer or option          */
  RIGA_ERR_NOT_SPD = -2,       /* a Cholesky pivot of Q(sigma) was <= 0       */
  RIGA_ERR_HIP = -3,           /* a HIP runtime call failed                    */
  RIGA_ERR_OOM = -4,           /* device allocation failed                     */
  RIGA_ERR_STATE = -5,         /* call out of order (e.g. eigs before factor)  */
  RIGA_ERR_SCRATCH = -6,       /* riga_solve_q_noalloc: the solve needs more
                                  than RIGA_NOALLOC_SCRATCH_BYTES of workspace */
  RIGA_WARN_NOT_CONVERGED = 1, /* eigs stopped at maxit, or fewer than nev pairs
                                  meet eta <= 1e-10: nconv < nev               */
  RIGA_WARN_IR_STAGNATED = 2    /* riga_factor_mixed: the refinement missed its
                                  target; the handle holds an FP64 factor      */
} riga_status;

/* Discretisation (Sec. 3.1-3.3).
 *   p            B-spline degree, 1 <= p <= 8.
 *   ne           elements per direction on (0,1)^2, ne >= 2.
 *   hyper_every  0: maximum-continuity IGA (interior knots of multiplicity 1,
 *                C^{p-1}; Sec. 3.2).  s > 0: rIGA, knots at multiples of s/ne
 *                get multiplicity p, i.e. C^0 hyperplanes that cut the square
 *                into (ne/s)^2 macroelements (Sec. 3.3); ne % s == 0 required.
 *   leaf         nested-dissection boxes without an interior hyperplane are
 *                bisected at element interfaces until both sides are <= leaf
 *                elements (0 = default 8: measured fastest for the factor and
 *                the sweeps at degrees 3-4).  With s <= leaf the rIGA leaves
 *                are the macroelements.
 *   space        RIGA_SPACE_H1 (0): the scalar space S^{p,p} with homogeneous
 *                Dirichlet conditions (the first and last function removed
 *                in each direction).  RIGA_SPACE_HCURL (1): the curl-conforming
 *                space S^{p-1,p} x S^{p,p-1} of eq. HcurlBasis (Sec. 3.2), dofs
 *                [E_x..., E_y...] as in eq. HcurlControlVariables; rIGA
 *                hyperplanes reduce the continuity by k-1 = p-2 (knot
 *                multiplicity p-1: C^1 in degree p, C^0 in degree p-1; eq.
 *                DiscreteSpacesrIGA); the tangential component vanishes on
 *                the boundary (the degree-p factor loses its end functions).
 *                RIGA_SPACE_HCURL_FREE (2): the same space without boundary
 *                condition (the matrices of fig. MatPatterns).
 *                RIGA_SPACE_HDIV (3): the divergence-conforming space
 *                S^{p,p-1} x S^{p-1,p} of eq. HdivBasis (the curl-conforming
 *                one rotated by 90 degrees), the same hyperplanes and dof
 *                layout, for the vibroacoustic model of Sec. 2.2: a rigid
 *                wall (u.n = 0) removes the degree-p function of the normal
 *                direction that is nonzero on it, an absorbing wall (a bit of
 *                `walls`) keeps it; riga_assemble then forms, with rho = c =
 *                1 and damping->alpha, damping->beta the wall coefficients of
 *                eq. HdivStrong, K = int div u div v + alpha G, M = int u . v,
 *                C = beta G, G = int over the absorbing walls of (u.n)(v.n)
 *                (eq. HdivWeak).  Vector spaces
 *                need p >= 2 and are assembled with K = int rot u rot v,
 *                M = int u . v (rot u = du_y/dx - du_x/dy), C = alpha M +
 *                beta K; they support riga_factor, the solves, the
 *                undamped case (riga_factor_gep, riga_gep_slice) and
 *                riga_eigs at a complex target (riga_factor_complex), not
 *                riga_eigs at a real shift, riga_apply_op, riga_factor_mixed,
 *                an element damping field, a gyroscopic part, the adjoint
 *                or a forest. */
typedef struct {
  int p, ne, hyper_every, leaf;
  int space;
  int walls;   /* RIGA_SPACE_HDIV: absorbing walls, RIGA_WALL_* bits; 0 otherwise */
} riga_mesh;
#define RIGA_SPACE_H1 0
#define RIGA_SPACE_HCURL 1
#define RIGA_SPACE_HCURL_FREE 2
#define RIGA_SPACE_HDIV 3
#define RIGA_WALL_LEFT 1     /* x = 0 */
#define RIGA_WALL_RIGHT 2    /* x = 1 */
#define RIGA_WALL_BOTTOM 4   /* y = 0 */
#define RIGA_WALL_TOP 8      /* y = 1 */

/* Damping C = alpha M + beta K + sum_e c_e M_e (Rayleigh part plus an optional
 * per-element viscous field).  c_elem: device, ne*ne doubles indexed
 * e = ey*ne + ex, or NULL for none.  Read during riga_assemble and kept by
 * reference for riga_adjoint (the caller keeps it alive until then).          */
typedef struct {
  double alpha, beta;
  const double* c_elem;
} riga_damping;

/* Eigensolver options (Alg. 2 and Sec. 4.1.3).
 *   nev     requested eigenpairs nearest sigma, 1 <= nev < 2N.
 *   m       Krylov subspace size, nev + block <= m, m <= 2N, m + 2 block <= 256
 *           (0: max(2 nev, 20)).
 *   maxit   maximum number of restarts (0: 200).
 *   block   block size of the Krylov iteration, 1..4 (0: 2).  Blocks of 2 resolve
 *           the exact double eigenvalues of the x<->y symmetric square.
 *   tol     relative Ritz residual for convergence (0: 1e-12).
 *   seed    seed of the library's counter-based start block (used if v0 NULL).
 *   v0      device, 2N x block column-major start block, or NULL.
 *   flags   bit 0: launch every block step eagerly instead of replaying its
 *           captured HIP graph; bit 1: check every block step on the host (the
 *           path otherwise taken only after a device-detected breakdown);
 *           RIGA_EIGS_TOAR (bit 2): keep the Krylov basis in compact two-level
 *           form (see riga_eigs); RIGA_EIGS_CGS2 (bit 3): take both
 *           Gram--Schmidt passes of a block within its own step (three reads
 *           of the basis per step) instead of delaying the second pass to the
 *           next step (two reads; the default for blocks of 1 and 2 on the
 *           device path; larger blocks always take both passes in the step).
 *   keep    Ritz values kept at a Krylov-Schur restart (0: nev + (m - nev)/2;
 *           at least nev, at most m - block; extended to whole clusters).    */
typedef struct {
  int nev, m, maxit, block;
  double tol;
  uint64_t seed;
  const double* v0;
  int flags;
  int keep;
} riga_options;
#define RIGA_EIGS_TOAR 4
#define RIGA_EIGS_CGS2 8

typedef struct {
  int64_t n1d;          /* 1-D functions per direction after Dirichlet          */
  int64_t ndof;         /* N = n1d^2                                            */
  int64_t nnz;          /* structural nonzeros of K, M, C and Q                 */
  int64_t nnodes;       /* nodes of the nested-dissection tree                  */
  int64_t nleaves;      /* leaves (rIGA: macroelements)                         */
  int64_t height;       /* levels of the tree (leaves = level 0)                */
  int64_t max_front;    /* largest front (own + boundary dofs)                  */
  int64_t leaf_own;     /* largest number of dofs eliminated in one leaf        */
  int64_t factor_entries;   /* stored entries of the factor (dense fronts)      */
  double  factor_flops_dense; /* flops executed by the dense-front factorization */
  double  solve_bytes;  /* bytes of factor read by one forward+backward solve   */
  int64_t factor_nnz;   /* nnz(L) of the symbolic Cholesky of Q under the
                           elimination order used (diagonal included; no
                           dense-front zeros)                                  */
  double  factor_flops; /* algorithmic factorization flops of that order:
                           sum_j (c_j^2 + 2 c_j), c_j = off-diagonal nonzeros
                           of column j of L (the cost C_fa of eq. Cost)        */
  int64_t upd_len;      /* entries of the update vectors one right-hand side
                           passes up the tree in a forward sweep              */
} riga_info_t;

/* Phases of the per-phase counters in riga_stats_t (eq. Cost of Sec. 5.1 and
 * the operation sets of Alg. 2).                                             */
enum {
  RIGA_PHASE_ASSEMBLE = 0,  /* K, M, C values                                    */
  RIGA_PHASE_FACTOR = 1,    /* factorization of Q(sigma)  (N_fa C_fa)            */
  RIGA_PHASE_FB = 2,        /* forward/backward eliminations (N_fb C_fb)         */
  RIGA_PHASE_MV = 3,        /* products with sigma M + C and M (N_mv C_mv)       */
  RIGA_PHASE_VV = 4,        /* B-orthogonalisation products (N_vv C_vv)          */
  RIGA_PHASE_RESTART = 5,   /* basis recombination at restarts and Ritz vectors  */
  RIGA_PHASE_IR = 6,        /* FP64 residual products of the mixed refinement    */
  RIGA_PHASE_POST = 7,      /* M, C, K products and forms of the returned pairs  */
  RIGA_NPHASE = 8
};

typedef struct {
  int64_t n_it;         /* Krylov-Schur restarts performed (N_it)               */
  int64_t n_fb;         /* forward/backward solves (one per vector, N_fb)       */
  int64_t n_mv;         /* sparse matrix-vector products (N_mv)                 */
  int64_t n_vv;         /* length-N vector-vector products (N_vv)               */
  int64_t n_ir;         /* FP64 refinement sweeps of the mixed factor (per vector;
                           each is one residual product and one FP32 solve)    */
  double t_assemble_ms, t_factor_ms, t_eigs_ms;  /* last call, device time     */
  double t_host_ms;     /* host wall time of the last eigensolve between its
                           device steps: projected-matrix downloads, Ritz
                           values and restarts, uploads (the device waits)    */
  /* Algorithmic work of the last assemble / factor / eigs calls per phase
   * (RIGA_PHASE_*), not the bytes a profiler counts.  flops follow eq. Cost:
   * C_fa = the symbolic count of riga_info_t.factor_flops; C_fb = 4 nnz(L)
   * per vector; C_mv = 2 nnz(Q) per product; C_vv = 2 N per length-N product;
   * assembly is a lower-order term there and counts 0 flops.  bytes are the
   * minimum HBM traffic of this library's kernels for that work: assembly
   * writes the three value arrays (24 B per nonzero, plus 8 B per element of
   * a damping field); the factorization reads them and writes nnz(L) entries;
   * a sweep pass reads the stored inverse blocks once per block of
   * right-hand sides plus 16 B per dof and vector; a sum-factorised product
   * moves 16 B per dof, a sparse one 8 B per stored entry plus 16 B per dof;
   * a length-N product reads 8 B per dof; a restart reads and writes the
   * three bases once.                                                         */
  double bytes[RIGA_NPHASE];
  double flops[RIGA_NPHASE];
  double toar_drop;     /* compact basis (RIGA_EIGS_TOAR): the largest norm a
                           restart's compression of U left out, relative to
                           the compact basis (rounding level when the
                           compression is exact); 0 for the full basis        */
} riga_stats_t;

/* Build the discretisation (open knot vectors of eq. KnotsX with C^0
 * hyperplanes of multiplicity p for rIGA, Sec. 3.1-3.3) and the
 * nested-dissection plan whose separators are the rIGA hyperplanes (the
 * elimination of Sec. 5.2.1) on the host, and allocate device storage on
 * `device` (HIP ordinal).  hip_stream: a hipStream_t, or NULL for the default
 * stream.  *out receives the handle; RIGA_ERR_INVALID_ARG for a mesh outside
 * the limits of riga_mesh, RIGA_ERR_OOM when device memory runs out.         */
riga_status riga_create(riga_problem** out, const riga_mesh* mesh, int device, void* hip_stream);

/* Sizes of the discretisation and of the factor plan (host output):
 * dimensions of the spaces of Sec. 3.2-3.3 and of the nested-dissection tree
 * whose separators are the rIGA hyperplanes (Sec. 3.3), the stored factor
 * and the cost C_fa of eq. Cost (Sec. 5.2.1) for the elimination order used.
 * The symbolic count is computed on the host at the first call.              */
riga_status riga_info(const riga_problem* h, riga_info_t* info);

/* Host-only symbolic Cholesky of Q(sigma)'s sparsity for a mesh (Sec. 5.2.1,
 * eq. CostFactIGA / eq. CostFactrIGA are its asymptotics), under the
 * elimination order this library's plan uses; touches no device.
 *   ndof:     host, receives N (may be NULL).
 *   order:    host, N int64 or NULL: order[k] = the dof eliminated k-th.
 *   colcount: host, N int64 or NULL: nonzeros of column k of L (elimination
 *             position k; diagonal included).
 *   nnz_l, flops: host or NULL: sum of colcount, sum_k (c_k^2 + 2 c_k) with
 *             c_k = colcount[k] - 1.
 * Call once with order = colcount = NULL to size the arrays.                 */
riga_status riga_symbolic(const riga_mesh* mesh, int64_t* ndof, int64_t* order, int64_t* colcount,
                          int64_t* nnz_l, double* flops);

/* Assemble K, M and C on the device (Sec. 3.1; element integrals by the
 * (p+1)^2-point Gauss rule).  Invalidates an existing factorization.         */
riga_status riga_assemble(riga_problem* h, const riga_damping* damping);

/* As riga_assemble, with a skew-symmetric (gyroscopic) part added to the
 * damping: the model-problem remark after eq. HcurlQuadEig (Sec. 2.1) takes a
 * skew-Hermitian damping matrix, C = -C^T, whose QEP is gyroscopic with a
 * spectrum symmetric with respect to the imaginary axis.  Here the skew part
 * is real, the form of a constant vector g = (gx, gy):
 *   C = alpha M + beta K + sum_e c_e M_e + G,   G_ab = int B_a (g . grad B_b),
 * skew-symmetric on the Dirichlet space (on the identity geometry
 * G = gx M1 (x) S1 + gy S1 (x) M1 with s_ij = int B_i B_j', x fastest).
 * Q(sigma) is then nonsymmetric with a positive definite symmetric part for
 * sigma > 0: riga_factor factors it by LU without pivoting on the same tree
 * (two triangles per front, twice the factor storage), and riga_eigs polishes
 * each eigenvalue as the root of u^H Q(lam) u = 0 (the pencil is not
 * complex-symmetric).  gx = gy = 0 is riga_assemble.  Not with
 * riga_factor_mixed or riga_adjoint (RIGA_ERR_INVALID_ARG); a forest's
 * problems cannot take it.  gx, gy finite.                                   */
riga_status riga_assemble_gyroscopic(riga_problem* h, const riga_damping* damping, double gx, double gy);

/* Copy one assembled matrix out in CSR form: which = 0 K, 1 M, 2 C, 3 C^T
 * (values of the transpose on the same pattern; only after
 * riga_assemble_gyroscopic with a nonzero g, else RIGA_ERR_STATE).
 *   rowptr: host, ndof+1 int64;  col: host, nnz int32;  val: device, nnz
 *   doubles.  Rows are dofs, columns ascend within a row.  Any of the three
 *   pointers may be NULL to skip it.                                         */
riga_status riga_export_csr(riga_problem* h, int which, int64_t* rowptr, int32_t* col, double* val);

/* Factor Q(sigma) = sigma^2 M + sigma C + K = L L^T (sigma > 0 makes Q SPD;
 * Sec. 4.2 and line 2 of Alg. 2) by a multifrontal Cholesky over the
 * nested-dissection tree whose separators are the rIGA hyperplanes.
 * On RIGA_ERR_NOT_SPD, *bad_pivot (if not NULL) receives the dof whose pivot
 * failed, else -1.                                                           */
riga_status riga_factor(riga_problem* h, double sigma, int64_t* bad_pivot);

/* A complex target sigma = sigma_re + i sigma_im (sigma_im > 0) inside the
 * complex spectrum region of interest (the target shift of Alg. 2, Sec. 4.1.1
 * with a complex shift).  Q(sigma) = R + iJ with R = (a^2 - b^2) M + a C + K,
 * J = b (2a M + C) (a = sigma_re, b = sigma_im) is factored in the real form
 * of -i Q(sigma) = J - iR on two unknowns per dof,
 *   [[J, R], [-R, J]]  (dof d: unknowns 2d = Re, 2d + 1 = Im),
 * by Gaussian elimination without pivoting on the same nested-dissection tree
 * (each front holds a dof's two unknowns together; the LU fronts of
 * riga_assemble_gyroscopic).  Its symmetric part is J (x) I, so the pivots are
 * positive when J is positive definite: C symmetric positive semidefinite
 * and 2a M + C positive definite (e.g. a >= 0 with alpha > 0).  Requires a
 * symmetric damping (riga_assemble), one problem (not a forest); any space,
 * including the curl-conforming ones, whose QEP riga_eigs then solves.
 * Afterwards riga_eigs runs on the real part of the shift-and-invert operator
 * (Parlett and Saad's real-part operator), Re S(sigma) = (S(sigma) +
 * S(conj sigma)) / 2, whose eigenvectors are the pencil's with the values
 *   psi(lam) = (1/(lam - sigma) + 1/(lam - conj sigma)) / 2,
 * and returns the nev eigenvalues of largest |psi| (near sigma or conj sigma,
 * in conjugate pairs); each is the root of u^T Q(lam) u = 0 whose psi is
 * nearest the Ritz value.  An eigenvalue on the circle |lam - a| = b has a
 * real psi shared with its conjugate and is resolved only as a pair.
 * Not with RIGA_EIGS_TOAR (RIGA_ERR_INVALID_ARG), riga_solve_q, riga_solve_q_noalloc,
 * riga_apply_op, riga_autotune or riga_time_kernel (RIGA_ERR_STATE: they use a real
 * factor); riga_solve_q_complex solves with the complex factor.  riga_adjoint
 * takes the returned pairs like any others.  The second factor (four times the entries of a real
 * Cholesky factor of the space, two triangles) and its workspace are
 * allocated at the first call and kept.  On RIGA_ERR_NOT_SPD, *bad_pivot
 * receives the dof of the failed pivot.  Synchronises.  riga_assemble,
 * riga_factor and riga_factor_gep end the complex mode.                     */
riga_status riga_factor_complex(riga_problem* h, double sigma_re, double sigma_im, int64_t* bad_pivot);

/* Q(sigma) x = b with the complex factor of riga_factor_complex.
 *   b, x: device, ndof x nrhs complex, interleaved (re, im), column-major
 *         (column stride 2 ndof doubles); nrhs >= 1; x must not alias b.
 * RIGA_ERR_STATE without a complex factor.  Asynchronous on the handle's
 * stream.                                                                   */
riga_status riga_solve_q_complex(riga_problem* h, int nrhs, const double* b, double* x);

/* Largest number of refinement sweeps per solve of a mixed factor.          */
#define RIGA_IR_MAX 10

/* Mixed-precision variant of riga_factor (the shift-and-invert factorization
 * of Sec. 4.2 / Alg. 2 with a reduced-precision factor and FP64 iterative
 * refinement).  Fronts of the tree levels below the top `fp64_levels` levels
 * (by height; 0 means 1, i.e. the root separator only) are factored in FP32
 * (FP32 MFMA products and accumulation) and stored in FP32; the top levels are
 * FP64.  Every later solve (riga_solve_q, riga_apply_op, the operator inside
 * riga_eigs) becomes x_0 = Q~^{-1} b, x_k = x_{k-1} + Q~^{-1}(b - Q x_{k-1}),
 * k = 1..ir_sweeps, with FP64 residuals of Q(sigma) (its values are kept
 * beside K, M, C) and FP64 sweep arithmetic over the FP32 blocks.
 *   ir_sweeps  0..RIGA_IR_MAX, or -1: chosen here from a refined solve of a
 *              seeded right-hand side: the fewest sweeps whose relative
 *              residual ||b - Q x_k|| / ||b|| is <= ir_tol, but never more
 *              than the point after which one more sweep would reduce it by
 *              less than a factor 4 (ir_tol = 0: that point).
 *   ir_tol     >= 0: the residual target of that calibration solve.
 * Stagnation: with ir_sweeps = -1, if the chosen count leaves the calibration
 * residual above ir_tol (above 1e-10 when ir_tol = 0), or with a fixed
 * ir_sweeps and ir_tol > 0, if that count leaves it above ir_tol, the FP32
 * factor is too weak for the refinement: Q(sigma) is factored again in FP64
 * (as riga_factor) and RIGA_WARN_IR_STAGNATED is returned; riga_ir_sweeps then
 * reports -1.  A fixed ir_sweeps with ir_tol = 0 is taken as given.
 *   ir_hist    host, RIGA_IR_MAX+1 doubles, or NULL: ||b - Q x_k|| / ||b|| for
 *              k = 0..RIGA_IR_MAX of that calibration solve (written whenever
 *              not NULL).
 *   bad_pivot  as for riga_factor.
 * Synchronises.  riga_factor switches the handle back to FP64.  Device memory
 * for the FP32 blocks (half the size of the FP64 factor) and the Q values is
 * allocated at the first call and kept.                                      */
riga_status riga_factor_mixed(riga_problem* h, double sigma, int fp64_levels, int ir_sweeps, double ir_tol,
                              double* ir_hist, int64_t* bad_pivot);

/* Refinement sweeps per solve of the current factor (-1 for an FP64 factor). */
riga_status riga_ir_sweeps(const riga_problem* h, int* sweeps);

/* x = Q(sigma)^{-1} b by the forward and backward sweeps of the factor
 * (Sec. 5.2.2).  b, x: device, ndof x nrhs column-major, 1 <= nrhs <= 4;
 * x may alias b.                                                             */
riga_status riga_solve_q(riga_problem* h, int nrhs, const double* b, double* x);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): riga_solve_q
 * with the same kernels, whose workspace (the forward sweep's result, the
 * update vectors passed up the tree and, for a mixed factor, the refinement's
 * iterate, residual and correction) lives in one static device array of
 * RIGA_NOALLOC_SCRATCH_BYTES per GPU instead of the handle's buffers.  The
 * call allocates nothing and queues its work like riga_solve_q.
 *   Needed workspace: 8 nrhs (ndof + upd_len) bytes for an FP64 factor and
 *   8 nrhs (4 ndof + upd_len) for a mixed one (ndof, upd_len from riga_info);
 *   a larger need returns RIGA_ERR_SCRATCH before anything is queued.
 * The array of a GPU is shared by every call on it and keeps the last call's
 * contents (a solve writes every entry before reading it): calls that overlap
 * on one GPU (several host threads, or several streams in flight) race.  The
 * device address of the array is looked up once per GPU, on the first call
 * there; the array lives until the process ends.                           */
#define RIGA_NOALLOC_SCRATCH_BYTES (64ull << 20)
riga_status riga_solve_q_noalloc(riga_problem* h, int nrhs, const double* b, double* x);

/* r = (A - sigma B)^{-1} B v for the companion pencil of eq. Linearization,
 * applied blockwise as in eq. BlockOperatorVector:
 *   r_u = -Q(sigma)^{-1} (sigma M v_u + C v_u + M v_l),  r_l = sigma r_u + v_u.
 * v, r: device, 2*ndof x nvec column-major (upper half u, lower half l),
 * 1 <= nvec <= 4; r must not alias v.                                        */
riga_status riga_apply_op(riga_problem* h, int nvec, const double* v, double* r);

/* The nev eigenpairs of the QEP nearest sigma (Alg. 2): block Krylov-Schur on
 * the shift-and-invert operator with B-orthogonal (CGS2) bases.  After
 * riga_factor_complex: the nev of largest |psi| on the real part of the
 * operator, in psi order (decreasing |psi|, ties by decreasing Im, then Re);
 * on a vector space only then.
 * With opt->flags & RIGA_EIGS_TOAR the basis is kept in the compact two-level
 * form V = [U Q1; U Q2] of the second-order Arnoldi methods (SOAR, cited in
 * Sec. 4.2.1): the lower block of the operator's image is sigma r_u + v_u
 * (eq. BlockOperatorVector), so every upper and lower block lies in the span
 * of one N x r orthonormal U (r = basis columns + block), and the long-vector
 * work of a step reads U alone (one N x r array instead of three N x k ones).
 * The inner product is then the Euclidean one of the 2N-space; the returned
 * pairs are computed, polished and checked as above.  m + 2 block <= 254.  A
 * case the compact form cannot run (a start block without full rank, a
 * breakdown) is solved with the full basis instead.
 *   lam: host, 2*nev doubles (re, im) in canonical order: increasing
 *        |lam - sigma|, ties (relative 1e-9) by decreasing Im, then Re.
 *   X:   device, ndof x nev complex (interleaved re, im), column k the
 *        eigenvector of lam_k normalised to u^H M u = 1 with an entry of
 *        largest modulus real positive (among entries tied up to rounding, the
 *        smallest dof); or NULL.
 *   eta: host, nev scaled residuals
 *        ||Q(lam)u|| / ((|lam|^2 ||M||_1 + |lam| ||C||_1 + ||K||_1) ||u||), or NULL.
 *   nconv: host, number of converged pairs returned in order.
 * RIGA_WARN_NOT_CONVERGED if maxit was reached first.                        */
riga_status riga_eigs(riga_problem* h, const riga_options* opt, double* lam, double* X,
                      double* eta, int* nconv);

/* Gradient of a real function L(lam_1..lam_nev) with respect to the per-element
 * damping field, for C = alpha M + beta K + sum_e c_e M_e.  For the
 * complex-symmetric pencil the left eigenvector is conj(u), so
 *   d lam_k / d c_e = -lam_k u_k^T M_e u_k / u_k^T (2 lam_k M + C) u_k
 * (unconjugated transposes; valid for simple eigenvalues), and
 *   grad_c[e] = sum_k dL/dRe(lam_k) Re(d lam_k/d c_e) + dL/dIm(lam_k) Im(d lam_k/d c_e).
 *   lam:     host, 2*nev doubles (re, im), e.g. from riga_eigs.
 *   X:       device, ndof x nev complex interleaved eigenvectors (any scaling).
 *   dL_dlam: host, 2*nev doubles (dL/dRe lam_k, dL/dIm lam_k).
 *   grad_c:  device, ne*ne doubles, e = ey*ne + ex.
 * Requires riga_assemble (the element tables); synchronises.                */
riga_status riga_adjoint(riga_problem* h, int nev, const double* lam, const double* X, const double* dL_dlam,
                         double* grad_c);

/* Operation counters of the cost model of Sec. 5.1 (eq. Cost) and phase times. */
riga_status riga_stats(const riga_problem* h, riga_stats_t* stats);

/* Measurement hook: time `reps` repetitions of one kernel family over all
 * tree levels with HIP events on the handle's stream (synchronises).
 *   which = 0  forward-sweep kernel, 1  backward-sweep kernel (nrhs vectors),
 *           2  front-factorization kernel (re-factors Q(sigma) in place).
 *   avg_ms            average duration of one launch (one tree level)
 *   work_per_launch   algorithmic work of one launch averaged over the levels:
 *                     bytes for the sweeps (factor entries read, lower triangle
 *                     of L_oo^{-1} and the boundary block, plus the vectors),
 *                     flops for the factorization (dense fronts).
 *   launches          launches per repetition (tree levels), may be NULL.
 * Requires a factored handle.                                                */
riga_status riga_time_kernel(riga_problem* h, int which, int nrhs, int reps, double* avg_ms,
                             double* work_per_launch, int* launches);

/* Autotuner of the sweep tile shapes (waves per 64-row task x 16-byte column
 * groups each wave keeps in flight; sweep layouts of Sec. 5.2.2's forward and
 * backward eliminations): every tree level and direction is timed with each
 * compiled shape on this handle's factor with nrhs right-hand sides (reps
 * launches each), and the fastest is kept for all later solves.  Choices are
 * cached in the process per device architecture, tree-level structure,
 * precision and nrhs, so a second handle of the same shape reuses them.
 * before_ms / after_ms (host, or NULL): one full forward+backward solve with
 * the previous and with the chosen shapes.  Requires a factored handle;
 * synchronises.                                                              */
riga_status riga_autotune(riga_problem* h, int nrhs, int reps, double* before_ms, double* after_ms);

/* The sweep shape chosen per tree level (host arrays of `height` ints, or
 * NULL) and the number of levels.                                            */
riga_status riga_sweep_shapes(const riga_problem* h, int* fwd, int* bwd, int* levels);

/* Host-only self-test of the dense small eigensolver used for the Ritz values
 * (Rayleigh-Ritz on the projected matrix, eq. ArnoldiRitz): a is n x n real
 * column-major (host); on return w holds the n eigenvalues (re, im pairs) and
 * resid the max ||a y - w y|| / ||a|| over the computed eigenvectors.  Touches
 * no device.                                                                 */
riga_status riga_selftest_small_eig(int n, const double* a, double* w, double* resid);

/* Host-only self-test of the Krylov--Schur restart's reordering (Sec. 4.1.3:
 * the kept Ritz values are moved to the top of the real Schur form by
 * exchanges of adjacent 1x1 / 2x2 blocks).  a: n x n real column-major
 * (host).  The nkeep eigenvalues of largest modulus (extended to every value
 * of equal modulus, so conjugate pairs stay whole) are kept.  On return r is
 * the kept dimension, w[0 .. 2r) the eigenvalues of the leading r x r block
 * (re, im pairs), resid the larger of max|a Q_r - Q_r T_rr| / max|a| and
 * max|Q_r^T Q_r - I|, real_path 1 when the real reordering was used.
 * RIGA_WARN_NOT_CONVERGED when the Schur iteration failed or an exchange was
 * ill conditioned (the solver then falls back to the complex form).  Touches
 * no device.                                                                 */
riga_status riga_selftest_schur_restart(int n, const double* a, int nkeep, int* r, double* w, double* resid,
                                        int* real_path);

/* Host-only self-test of the compression of the compact (TOAR) basis at a
 * restart: an orthonormal W (r x rp) whose range holds the columns of A (r x
 * nc, column-major, host) by Householder QR with column pivoting.  On return
 * W (host, r x rp) and *drop = the largest norm left outside range(W) after
 * rp pivots relative to the largest column norm of A (rounding level when
 * rank(A) <= rp).  Touches no device.                                        */
riga_status riga_selftest_range_basis(int r, int nc, const double* a, int rp, double* w, double* drop);

/* ---- Undamped problem: K u = mu M u with spectrum slicing --------------------
 * With C = 0 the QEP of eq. QuadEig reduces to the Hermitian definite pencil
 * K u = mu M u (lam^2 = -mu, the non-conductive case), whose eigenvalues are
 * real and positive.  Sec. 4.1.4 (spectrum slicing): for K - s M = L D L^T,
 * Sylvester's law of inertia makes the number of negative pivots the number of
 * eigenvalues below s, so an interval splits into slices of known counts; each
 * slice is solved by the Lanczos recurrence (the Lanczos remark of Sec. 4.1.2:
 * the projected matrix of this operator is symmetric) on the shift-and-invert
 * operator (K - s M)^{-1} M of a shift inside it, with Krylov--Schur (thick)
 * restarts (Sec. 4.1.3).  Requires riga_assemble; its damping is ignored.   */

/* Factor K - shift M over the nested-dissection tree in the signed form
 * L S L^T (LDL^T without pivoting, S = diag(+-1) folded into L; any real
 * shift) and return *neg_count = the number of negative pivots = the number of
 * eigenvalues mu < shift, with multiplicity (neg_count host, or NULL).
 * RIGA_ERR_NOT_SPD when a pivot is zero or NaN (shift on an eigenvalue to
 * working precision), with *bad_pivot (host, or NULL) as for riga_factor.
 * Synchronises.  Afterwards riga_solve_q and riga_solve_q_noalloc solve with
 * K - shift M; riga_eigs and riga_apply_op return RIGA_ERR_STATE until
 * riga_factor or riga_factor_mixed factors Q(sigma) again.                   */
riga_status riga_factor_gep(riga_problem* h, double shift, int64_t* neg_count, int64_t* bad_pivot);

/* Every eigenvalue of K u = mu M u in [a, b) (a < b) with its eigenvector, by
 * spectrum slicing:
 *   1. count = nu(b) - nu(a) from two signed factorizations;
 *   2. a slice holding more than max_slice eigenvalues (0: 40; >= 2) is
 *      bisected at its midpoint, whose count costs one factorization; on a
 *      vector space (whose gradients are a null space of large multiplicity)
 *      a slice [l, r) holding eigenvalues is also bisected until
 *      r - l <= l / 2, so that the null space's operator value -1/s stays
 *      well below the slice's own (a > 0 there: a <= 0 counts the whole null
 *      space);
 *   3. each slice [l, r) with k > 0 eigenvalues is factored at its midpoint s
 *      (moved by 1e-9 relative if a pivot vanishes) and solved by block Lanczos
 *      (opt->block, 0: 2; opt->tol, opt->maxit, opt->seed as for riga_eigs;
 *      opt->nev, opt->m and opt->keep are chosen per slice: the k + 2 values of
 *      theta = 1/(mu - s) of largest modulus, subspace max(2 (k + 2), 20)); the
 *      converged values with mu in [l, r) are returned.  On a vector space
 *      Ritz values with |mu| <= 1e-6 |s| (the null space) are neither counted
 *      among the k + 2 nor kept at restarts.
 *   cap    room (pairs) in mu / U / resid; count > cap gives RIGA_ERR_INVALID_ARG
 *          with *count written.
 *   mu     host, cap doubles: the eigenvalues, ascending: with U, the Rayleigh
 *          quotients u^T K u / u^T M u of the returned vectors (error quadratic
 *          in theirs); without, the Ritz values s + 1/theta, whose error grows
 *          as (mu - s)^2 away from the slice's shift.
 *   U      device, ndof x cap column-major, or NULL: M-orthonormal eigenvectors.
 *   resid  host, cap doubles, or NULL (needs U): ||K u - mu M u||_2 /
 *          ((||K||_1 + |mu| ||M||_1) ||u||_2).
 *   count  host: nu(b) - nu(a).   found: host: pairs returned.
 *   stats  host, 4 int64 or NULL: factorizations, slices, operator applications,
 *          restarts.
 * RIGA_WARN_NOT_CONVERGED when a slice returns fewer pairs than its count.
 * Synchronises; leaves the handle factored at the last slice's shift.        */
riga_status riga_gep_slice(riga_problem* h, double a, double b, int max_slice, const riga_options* opt, int cap,
                           double* mu, double* U, double* resid, int64_t* count, int* found, int64_t* stats);

/* ---- Batched form -----------------------------------------------------------
 * The paper solves one problem at a time; every problem here follows the
 * single-problem method above (Alg. 2 on the pencil of eq. Linearization with
 * the factorization of Sec. 5.2.1), and the batching is this library's own
 * execution form.
 * Many independent problems of different sizes (degree, mesh, hyperplane
 * spacing, damping, shift) solved together: the nested-dissection trees are
 * merged into one forest, so each factorization level and each sweep is one
 * set of launches for all problems, and the Krylov--Schur iterations of all
 * problems run in lockstep, one captured HIP graph per block step of every
 * problem.  Each problem follows exactly the single-problem method above
 * (same operator, orthogonalisation, restart and convergence test).          */
typedef struct riga_batch riga_batch;

/* n >= 1 problems; meshes: host array of n (as for riga_create).  Builds every
 * plan on the host and allocates the forest on `device`.                     */
riga_status riga_batch_create(riga_batch** out, int n, const riga_mesh* meshes, int device, void* hip_stream);

/* Total dofs and (if dof_offsets is not NULL, host n+1) the first dof of every
 * problem in the forest numbering: problem p owns rows
 * [dof_offsets[p], dof_offsets[p+1]).                                         */
riga_status riga_batch_info(const riga_batch* bh, int64_t* total_dofs, int64_t* dof_offsets);

/* Assemble every problem; damping: host array of n (c_elem device or NULL).    */
riga_status riga_batch_assemble(riga_batch* bh, const riga_damping* damping);

/* Factor Q_p(sigma_p) of every problem; sigmas: host, n values > 0.  On
 * RIGA_ERR_NOT_SPD, bad_pivot (host n, or NULL) holds the failing dof of the
 * problem it occurred in (-1 elsewhere).                                     */
riga_status riga_batch_factor(riga_batch* bh, const double* sigmas, int64_t* bad_pivot);

/* The opt->nev eigenpairs nearest sigma_p of every problem (options as for
 * riga_eigs; opt->v0 must be NULL: the start blocks come from the library's
 * generator; 2 N_p >= m for every problem).
 *   lam:   host, n * 2 * nev doubles, problem p at lam + 2 nev p, canonical order.
 *   X:     device, 2 * nev * total_dofs doubles or NULL: problem p's block at
 *          X + 2 nev dof_offsets[p], column k at + 2 k N_p, normalised as in
 *          riga_eigs.
 *   eta:   host, n * nev scaled residuals, or NULL.
 *   nconv: host, n counts.
 * A problem whose block step broke down (an exact invariant subspace) is
 * solved again on its own with the host-checked path.  Synchronises.
 * RIGA_WARN_NOT_CONVERGED if any problem has nconv < nev.                     */
riga_status riga_batch_eigs(riga_batch* bh, const riga_options* opt, double* lam, double* X, double* eta,
                            int* nconv);

/* riga_autotune for the forest of the batch (shapes chosen per tree level
 * across all problems).                                                      */
riga_status riga_batch_autotune(riga_batch* bh, int nrhs, int reps, double* before_ms, double* after_ms);

/* Phase times and counters of the last calls (n_it: lockstep cycles; n_fb:
 * vectors through the sweeps summed over problems); n_resolved (or NULL): the
 * problems solved again one by one in the last riga_batch_eigs.              */
riga_status riga_batch_stats(const riga_batch* bh, riga_stats_t* stats, int* n_resolved);

void riga_batch_destroy(riga_batch* bh);

const char* riga_status_str(riga_status s);
void riga_destroy(riga_problem* h);

#ifdef __cplusplus
}
#endif
#endif /* RIGA_H */
