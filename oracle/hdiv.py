"""The divergence-conforming space S^{p,p-1} x S^{p-1,p} (Sec. 3.2, eq.
HdivBasis; rIGA: eq. DiscreteSpacesrIGA) on the unit square and the matrices
of the vibroacoustic QEP of Sec. 2.2 (eq. HdivWeak, eq. HdivQuadEig).

Oracle module: test infrastructure only.

Space: component x of the field is B^p_i(x) B^{p-1}_j(y), component y is
B^{p-1}_i(x) B^p_j(y), both degrees with hyperplane knots of multiplicity p-1
(as the curl-conforming space, of which this is the rotation by 90 degrees).
Walls, a bitmask `absorbing`: 1 left (x = 0), 2 right (x = 1), 4 bottom
(y = 0), 8 top (y = 1).  A rigid wall (bit clear) imposes u.n = 0: the
degree-p function of the normal direction that is nonzero on that wall (the
first at 0, the last at 1) is removed from the component normal to it; an
absorbing wall keeps it.  Dofs: all x components first (x fastest), then the
y components (eq. HcurlControlVariables' layout).

Forms (rho = c = 1; alpha, beta the wall coefficients of eq. HdivStrong):
    K = int div u div v + alpha int_{Gamma_A} (u.n)(v.n),
    C = beta int_{Gamma_A} (u.n)(v.n),
    M = int u . v,
the domain integrals by the (p+1) x (p+1) Gauss rule on every element, the
wall integrals by the (p+1)-point rule on every wall element, from the 2-D
vector basis.  On a wall the normal component u.n is u_x (x walls) or u_y
(y walls), the sign of n dropping out of the product.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .bspline import basis, gauss_legendre, knot_vector, n_functions
from .hcurl import _element_values

LEFT, RIGHT, BOTTOM, TOP = 1, 2, 4, 8


def spaces(p, ne, hyper_every, absorbing):
    """Knot vectors of the degree-p space B and the degree-(p-1) space A
    (multiplicity p-1 at the hyperplanes), and per component the kept
    functions of B in its normal direction: (kvA, kvB, nA, (x0, x1), (y0, y1))
    with x0..x1-1 the kept B functions of component x in x, y0..y1-1 those of
    component y in y."""
    kvA = knot_vector(p - 1, ne, hyper_every, mult=p - 1)
    kvB = knot_vector(p, ne, hyper_every, mult=p - 1)
    nA = n_functions(kvA, p - 1)
    nB = n_functions(kvB, p)
    x0 = 0 if absorbing & LEFT else 1
    x1 = nB if absorbing & RIGHT else nB - 1
    y0 = 0 if absorbing & BOTTOM else 1
    y1 = nB if absorbing & TOP else nB - 1
    return kvA, kvB, nA, (x0, x1), (y0, y1)


def assemble_hdiv(p, ne, hyper_every=0, absorbing=0, alpha=0.0, beta=0.0):
    """(K, M, C) in CSR; the stored pattern holds every pair of functions
    sharing an element (explicit zeros kept)."""
    kvA, kvB, nA, (x0, x1), (y0, y1) = spaces(p, ne, hyper_every, absorbing)
    nBx, nBy = x1 - x0, y1 - y0
    npts = p + 1
    fA, VA, DA, w = _element_values(kvA, p - 1, ne, npts)
    fB, VB, DB, _ = _element_values(kvB, p, ne, npts)
    base1 = nBx * nA
    N = base1 + nA * nBy
    W2 = np.outer(w, w)
    rows, cols, vk, vm = [], [], [], []
    for ey in range(ne):
        for ex in range(ne):
            loc = []   # (dof, ux[qy, qx], uy[qy, qx], div[qy, qx])
            for lb in range(p):                  # component x: B(x) A(y)
                gy = fA[ey] + lb
                for la in range(p + 1):
                    gx = fB[ex] + la
                    if not (x0 <= gx < x1):
                        continue
                    val = np.outer(VA[ey][:, lb], VB[ex][:, la])
                    dx = np.outer(VA[ey][:, lb], DB[ex][:, la])
                    loc.append(((gy) * nBx + gx - x0, val, np.zeros_like(val), dx))
            for lb in range(p + 1):              # component y: A(x) B(y)
                gy = fB[ey] + lb
                if not (y0 <= gy < y1):
                    continue
                for la in range(p):
                    gx = fA[ex] + la
                    val = np.outer(VB[ey][:, lb], VA[ex][:, la])
                    dy = np.outer(DB[ey][:, lb], VA[ex][:, la])
                    loc.append((base1 + (gy - y0) * nA + gx, np.zeros_like(val), val, dy))
            dofs = np.array([d for d, _, _, _ in loc])
            UX = np.stack([u for _, u, _, _ in loc])
            UY = np.stack([u for _, _, u, _ in loc])
            DV = np.stack([d for _, _, _, d in loc])
            Ke = np.einsum("aqr,bqr,qr->ab", DV, DV, W2)
            Me = np.einsum("aqr,bqr,qr->ab", UX, UX, W2) + np.einsum("aqr,bqr,qr->ab", UY, UY, W2)
            rows.append(np.repeat(dofs, len(dofs)))
            cols.append(np.tile(dofs, len(dofs)))
            vk.append(Ke.reshape(-1))
            vm.append(Me.reshape(-1))
    r = np.concatenate(rows); c = np.concatenate(cols)
    K = sp.coo_matrix((np.concatenate(vk), (r, c)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.concatenate(vm), (r, c)), shape=(N, N)).tocsr()
    G = wall_mass(p, ne, hyper_every, absorbing)
    for A in (K, M):
        A.sum_duplicates()
        A.sort_indices()
    g = _on_pattern(G, K)
    K.data = K.data + alpha * g
    C = K.copy()
    C.data = beta * g
    return K, M, C


def _on_pattern(G, P):
    """Values of the sparse G at the stored positions of P, in P's order
    (every entry of G must lie in the pattern: wall pairs share an element)."""
    G = G.tocsr()
    out = np.zeros(P.nnz)
    found = 0
    for i in range(P.shape[0]):
        gi = dict(zip(G.indices[G.indptr[i]:G.indptr[i + 1]], G.data[G.indptr[i]:G.indptr[i + 1]]))
        for k in range(P.indptr[i], P.indptr[i + 1]):
            if P.indices[k] in gi:
                out[k] = gi[P.indices[k]]
                found += 1
    assert found == G.nnz
    return out


def wall_mass(p, ne, hyper_every, absorbing):
    """G = int_{Gamma_A} (u.n)(v.n) over the absorbing walls, by the
    (p+1)-point Gauss rule on each wall element, from the 2-D basis evaluated
    on the wall (a degree-p B-spline of an open knot vector is 1 at its end
    for the end function and 0 for the others)."""
    kvA, kvB, nA, (x0, x1), (y0, y1) = spaces(p, ne, hyper_every, absorbing)
    nBx, nBy = x1 - x0, y1 - y0
    nB = n_functions(kvB, p)
    base1 = nBx * nA
    N = base1 + nA * nBy
    xg, wg = gauss_legendre(p + 1)
    h = 1.0 / ne
    G = sp.lil_matrix((N, N))
    pts = (np.arange(ne)[:, None] * h + (xg[None, :] + 1.0) * 0.5 * h).reshape(-1)
    wts = np.tile(wg * 0.5 * h, ne)
    VAw = basis(kvA, p - 1, pts)          # A functions along the wall
    end = {0: np.eye(nB)[0], 1: np.eye(nB)[-1]}   # B values at 0 and at 1
    for bit, comp, side in ((LEFT, 0, 0), (RIGHT, 0, 1), (BOTTOM, 1, 0), (TOP, 1, 1)):
        if not absorbing & bit:
            continue
        bval = end[side]
        dofs, vals = [], []
        if comp == 0:        # x walls: u.n = u_x = B_i(x_wall) A_j(y)
            for j in range(nA):
                for i in range(x0, x1):
                    if bval[i] != 0.0:
                        dofs.append(j * nBx + i - x0)
                        vals.append(bval[i] * VAw[:, j])
        else:                # y walls: u.n = u_y = A_i(x) B_j(y_wall)
            for j in range(y0, y1):
                if bval[j] == 0.0:
                    continue
                for i in range(nA):
                    dofs.append(base1 + (j - y0) * nA + i)
                    vals.append(bval[j] * VAw[:, i])
        V = np.stack(vals)
        Gl = np.einsum("aq,bq,q->ab", V, V, wts)
        for a, da in enumerate(dofs):
            for b, db in enumerate(dofs):
                if Gl[a, b] != 0.0:
                    G[da, db] += Gl[a, b]
    return G.tocsr()


def rotation(p, ne, hyper_every):
    """The signed permutation P with u_div = P u_curl for v = (u_y, -u_x) on
    the rigid / perfect-conductor spaces (all walls rigid here): the
    divergence-conforming component x is the curl-conforming component y, and
    component y is minus component x.  K_div = P K_curl P^T, M_div = P M_curl
    P^T (div v = rot u, |v| = |u|)."""
    kvA, kvB, nA, (x0, x1), (y0, y1) = spaces(p, ne, hyper_every, 0)
    nBx, nBy = x1 - x0, y1 - y0
    ncx = nA * nBy          # curl component x: A(x) B(y), nA x nB
    N = 2 * nA * nBx
    rows, cols, vals = [], [], []
    for k in range(nBx * nA):      # div comp x (B(x) A(y)) <- curl comp y (same layout) at ncx + k
        rows.append(k); cols.append(ncx + k); vals.append(1.0)
    for k in range(nA * nBy):      # div comp y (A(x) B(y)) <- -curl comp x (same layout) at k
        rows.append(nBx * nA + k); cols.append(k); vals.append(-1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
