"""The curl-conforming space S^{p-1,p} x S^{p,p-1} (Sec. 3.2, eq. HcurlBasis;
rIGA: eq. DiscreteSpacesrIGA) on the unit square and its Maxwell matrices.

Oracle module: test infrastructure only.

Space: component x of the field is B^{p-1}_i(x) B^p_j(y), component y is
B^p_i(x) B^{p-1}_j(y).  Maximum continuity is k = p-1 in the degree-p
direction and k-1 in the degree-(p-1) one; rIGA lowers both by k-1 = p-2 at
the hyperplanes, so both degrees carry knots of multiplicity p-1 there (C^1
and C^0).  Boundary conditions: "pec" removes the first and last degree-p
function in each direction (the tangential component vanishes on the
boundary, the perfect-conductor condition of the Maxwell remark of Sec. 2.1);
"free" keeps all functions (the matrices of fig. MatPatterns).  Dofs: all x
components first (x fastest), then the y components (eq.
HcurlControlVariables).

Forms (identity geometry, Sec. 3.2 maps are identities):
    K_ab = int rot u_a rot u_b,  rot u = du_y/dx - du_x/dy,
    M_ab = int u_a . u_b,        C = alpha M + beta K,
by the (p+1) x (p+1) Gauss rule on every element from the 2-D vector basis.

Routes:
  * assemble_hcurl -- the element assembly above;
  * grad_matrix    -- the discrete gradient from the scalar space S^{p,p}
                      (same knots) into this space, from the derivative
                      formula of B-splines (no integration): the exactness of
                      the de Rham sequence gives K G = 0;
  * maxwell_closed -- the nonzero eigenvalues of K u = mu M u: by the tensor
                      structure of the sequence they are the sums nu_a + nu_b
                      of 1-D values, nu over {0} and the eigenvalues of the
                      Dirichlet 1-D pencil of the degree-p space (pec), or over
                      the positive eigenvalues of its Neumann pencil (free),
                      excluding nu_a = nu_b = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .bspline import basis, basis_deriv, gauss_legendre, knot_vector, n_functions


def _element_values(kv, q, ne, npts):
    """Per element: the index of its first nonzero degree-q function and the
    values / derivatives of its q+1 functions at the npts Gauss points."""
    xg, wg = gauss_legendre(npts)
    h = 1.0 / ne
    pts = (np.arange(ne)[:, None] * h + (xg[None, :] + 1.0) * 0.5 * h).reshape(-1)
    V = basis(kv, q, pts)
    Dv = basis_deriv(kv, q, pts)
    first = np.zeros(ne, dtype=np.int64)
    Bv = np.zeros((ne, npts, q + 1))
    Bd = np.zeros((ne, npts, q + 1))
    for e in range(ne):
        mid = (e + 0.5) * h
        k = int(np.searchsorted(kv, mid, side="right") - 1)
        first[e] = k - q
        Bv[e] = V[e * npts:(e + 1) * npts, k - q:k + 1]
        Bd[e] = Dv[e * npts:(e + 1) * npts, k - q:k + 1]
    return first, Bv, Bd, wg * 0.5 * h


def spaces(p, ne, hyper_every, pec):
    """(kvA, kvB, offB, nA, nB): knot vectors of the degree-(p-1) space A and
    the degree-p space B (hyperplane multiplicity p-1), B's first kept
    function and both dimensions."""
    kvA = knot_vector(p - 1, ne, hyper_every, mult=p - 1)
    kvB = knot_vector(p, ne, hyper_every, mult=p - 1)
    nA = n_functions(kvA, p - 1)
    offB = 1 if pec else 0
    nB = n_functions(kvB, p) - 2 * offB
    return kvA, kvB, offB, nA, nB


def assemble_hcurl(p, ne, hyper_every=0, pec=True, alpha=0.0, beta=0.0):
    """(K, M, C) in CSR (explicit zeros kept: M vanishes between the two
    components but the stored pattern holds every pair sharing an element)."""
    kvA, kvB, offB, nA, nB = spaces(p, ne, hyper_every, pec)
    npts = p + 1
    fA, VA, DA, w = _element_values(kvA, p - 1, ne, npts)
    fB, VB, DB, _ = _element_values(kvB, p, ne, npts)
    base1 = nA * nB
    W2 = np.outer(w, w)                          # [qy, qx]
    rows, cols, vk, vm = [], [], [], []
    for ey in range(ne):
        for ex in range(ne):
            # local basis: component 0 dofs (la, lb): A_la(x) B_lb(y); component 1: B_la(x) A_lb(y)
            loc = []       # (global dof, ux[qy,qx], uy[qy,qx], rot[qy,qx])
            for lb in range(p + 1):
                gy = fB[ey] + lb - offB
                if gy < 0 or gy >= nB:
                    continue
                for la in range(p):
                    gx = fA[ex] + la
                    val = np.outer(VB[ey][:, lb], VA[ex][:, la])          # [qy, qx]
                    dy = np.outer(DB[ey][:, lb], VA[ex][:, la])
                    loc.append((gy * nA + gx, val, np.zeros_like(val), -dy))
            for lb in range(p):
                gy = fA[ey] + lb
                for la in range(p + 1):
                    gx = fB[ex] + la - offB
                    if gx < 0 or gx >= nB:
                        continue
                    val = np.outer(VA[ey][:, lb], VB[ex][:, la])
                    dx = np.outer(VA[ey][:, lb], DB[ex][:, la])
                    loc.append((base1 + gy * nB + gx, np.zeros_like(val), val, dx))
            dofs = np.array([d for d, _, _, _ in loc])
            UX = np.stack([u for _, u, _, _ in loc])
            UY = np.stack([u for _, _, u, _ in loc])
            R = np.stack([r_ for _, _, _, r_ in loc])
            Ke = np.einsum("aqr,bqr,qr->ab", R, R, W2)
            Me = np.einsum("aqr,bqr,qr->ab", UX, UX, W2) + np.einsum("aqr,bqr,qr->ab", UY, UY, W2)
            rows.append(np.repeat(dofs, len(dofs)))
            cols.append(np.tile(dofs, len(dofs)))
            vk.append(Ke.reshape(-1))
            vm.append(Me.reshape(-1))
    N = base1 + nA * nB
    r = np.concatenate(rows); c = np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(vk), (r, c)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.concatenate(vm), (r, c)), shape=(N, N)).tocsr()
    for A in (K, M):
        A.sum_duplicates()
        A.sort_indices()
    C = K.copy()
    C.data = alpha * M.data + beta * K.data
    return K, M, C


def grad_matrix(p, ne, hyper_every=0, pec=True):
    """G (N_curl x N_scalar): the coefficients of grad(B_i(x) B_j(y)) in this
    space, for the scalar space S^{p,p} on the same degree-p knot vector
    (Dirichlet when pec).  d/dx B^p_i = p (B^{p-1}_i / (t_{i+p} - t_i) -
    B^{p-1}_{i+1} / (t_{i+p+1} - t_{i+1})) on the same knots t, and B^{p-1}_i
    on t is function i - 1 of the degree-(p-1) knot vector (t without its
    first and last knot); terms with a zero denominator vanish."""
    kvA, kvB, offB, nA, nB = spaces(p, ne, hyper_every, pec)
    t = kvB
    nall = n_functions(kvB, p)

    def dcoef(i):
        out = []
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0:
            out.append((i - 1, p / d1))
        if d2 > 0:
            out.append((i, -p / d2))
        return [(a, v) for a, v in out if 0 <= a < nA]

    base1 = nA * nB
    rows, cols, vals = [], [], []
    for j in range(nB):
        for i in range(nB):
            s = j * nB + i          # scalar dof (kept functions i + offB, j + offB)
            fi, fj = i + offB, j + offB
            # x component: (dB_fi/dx)(x) B_fj(y) = sum_a c_a A_a(x) B_fj(y)
            for a, v in dcoef(fi):
                rows.append(j * nA + a); cols.append(s); vals.append(v)
            # y component: B_fi(x) (dB_fj/dy)(y) = sum_b c_b B_fi(x) A_b(y)
            for b, v in dcoef(fj):
                rows.append(base1 + b * nB + i); cols.append(s); vals.append(v)
    assert nall - 2 * offB == nB
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nA * nB, nB * nB))


def pencil_1d(p, ne, hyper_every=0, pec=True):
    """Dense 1-D stiffness and mass matrices of the degree-p space with
    hyperplane multiplicity p-1 (pec: without its end functions)."""
    kvA, kvB, offB, nA, nB = spaces(p, ne, hyper_every, pec)
    fB, VB, DB, w = _element_values(kvB, p, ne, p + 1)
    nall = n_functions(kvB, p)
    K1 = np.zeros((nall, nall)); M1 = np.zeros((nall, nall))
    for e in range(ne):
        g = fB[e] + np.arange(p + 1)
        M1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, VB[e], VB[e])
        K1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, DB[e], DB[e])
    if pec:
        return K1[1:-1, 1:-1], M1[1:-1, 1:-1]
    return K1, M1


def maxwell_closed(p, ne, hyper_every, pec, a, b):
    """Every nonzero eigenvalue of K u = mu M u in [a, b) (a > 0), sorted, with
    multiplicity: nu_a + nu_b over ordered pairs of 1-D values (see the
    module docstring).  The 1-D values are Rayleigh quotients of LAPACK's
    eigenvectors (quadratic in the vectors' error)."""
    K1, M1 = pencil_1d(p, ne, hyper_every, pec)
    w, V = sla.eigh(K1, M1)
    rq = np.einsum("ik,ij,jk->k", V, K1, V) / np.einsum("ik,ij,jk->k", V, M1, V)
    nu = np.sort(rq)
    if pec:
        nu = np.concatenate([[0.0], nu])
    else:
        nu = nu[1:]          # the constant's zero
    out = []
    for x in nu:
        for y in nu:
            m = x + y
            if m == 0.0:
                continue
            if a <= m < b:
                out.append(m)
    return np.sort(np.asarray(out))


def null_dimension(p, ne, hyper_every, pec):
    """Multiplicity of the zero eigenvalue: the dimension of the gradients of
    the scalar space (n_B^2, minus the constants when free)."""
    _, _, _, nA, nB = spaces(p, ne, hyper_every, pec)
    return nB * nB if pec else nB * nB - 1
