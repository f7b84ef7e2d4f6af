"""Plain FP64 CPU oracle for the damped-wave QEP discretised with IGA / rIGA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this package; only the test-suite, the package smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code,
tables or constants with the HIP library and is written for a reader who has
the paper beside it: every function names the section or equation it follows.

What it computes is the *definition* of the result, not the paper's method:
the N_ev eigenvalues of the discrete QEP (K + lam C + lam^2 M) u = 0
(Sec. 4.2, eq. QuadEig) nearest the shift sigma, for a given B-spline space.
Shift-and-invert, linearisation, Arnoldi, restarting and multifrontal
factorisation are ways of reaching exactly this set faster.

Modules
    bspline   knot vectors (eq. KnotsX/KnotsY), Cox--de Boor (eq. BasisFunBi0/Bip),
              Gauss--Legendre rule
    space     1-D supports, dimension and sparsity counts (Sec. 3.2-3.3, fig. MatPatterns)
    assemble  K, M, C on the unit square, Dirichlet elimination, Q(sigma)
    eigen     dense companion-pencil QZ (eq. Linearization), Rayleigh-damping closed
              form, sparse shift-and-invert (eq. BlockOperatorVector), residual,
              canonical ordering
    adjoint   d lam / d c_e for a per-element damping field
    gep       the undamped pencil K u = mu M u: closed-form eigenvalues in an interval,
              dense solver, inertia counts (Sec. 4.1.4, spectrum slicing), residual
    hcurl     the curl-conforming space S^{p-1,p} x S^{p,p-1} (Sec. 3.2-3.3): element assembly
              of the curl-curl and mass matrices, the discrete gradient, the Maxwell
              eigenvalues as sums of 1-D values
    gyro      damping with a skew-symmetric (gyroscopic) part G_ab = int B_a (g . grad B_b):
              element assembly, the 1-D skew matrix, eigenvalues from the 1-D QEPs
              of the y-modes (gy = 0)
    hdiv      the divergence-conforming space S^{p,p-1} x S^{p-1,p} and the vibroacoustic QEP
              (Sec. 2.2): element assembly of div-div and mass matrices, the absorbing-wall
              integrals, the rotation to the curl-conforming space
    cshift    a complex target shift: the eigenvalues of largest |psi| for the real
              part of the shift-and-invert operator (closed forms on the scalar and
              curl-conforming spaces, ARPACK's real-part mode)
"""
