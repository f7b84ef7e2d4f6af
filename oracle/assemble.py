"""Galerkin matrices of the scalar damped-wave QEP on the unit square.

Oracle module: test infrastructure only.

Space: tensor-product B-splines B_i(x) B_j(y) (Sec. 3.1) on the identity
geometry, so the mappings of Sec. 3.2 reduce to the identity.  Forms:
    K_ab = int grad B_a . grad B_b,   M_ab = int B_a B_b,
    C    = alpha M + beta K + sum_e c_e M_e,
integrated element by element with the (p+1) x (p+1) Gauss--Legendre rule.
Homogeneous Dirichlet conditions are imposed by deleting the first and last
1-D function in each direction.  Dofs are lexicographic, x fastest:
dof(i, j) = j * n1d + i over the remaining functions.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp

from .bspline import basis, basis_deriv, gauss_legendre, knot_vector, n_functions


@functools.lru_cache(maxsize=16)
def _element_tables(p, ne, hyper_every):
    """Per element: index of the first of its p+1 nonzero functions, and the
    values / derivatives of those functions at the element's Gauss points.
    Cached per space; callers treat the arrays as read-only."""
    kv = knot_vector(p, ne, hyper_every)
    xg, wg = gauss_legendre(p + 1)
    h = 1.0 / ne
    first = np.zeros(ne, dtype=np.int64)
    B = np.zeros((ne, p + 1, p + 1))   # [element, gauss point, local function]
    D = np.zeros((ne, p + 1, p + 1))
    # every element's Gauss points in one call: the recursion acts pointwise,
    # so each point gets the same arithmetic as if evaluated on its own
    pts_all = (np.arange(ne)[:, None] * h + (xg[None, :] + 1.0) * 0.5 * h).reshape(-1)
    Ball_all = basis(kv, p, pts_all)
    Dall_all = basis_deriv(kv, p, pts_all)
    nl = p + 1
    for e in range(ne):
        a = e * h
        # the knot span holding the element: last knot index with t_k <= midpoint
        mid = a + 0.5 * h
        k = int(np.searchsorted(kv, mid, side="right") - 1)
        first[e] = k - p
        Ball = Ball_all[e * nl:(e + 1) * nl]
        Dall = Dall_all[e * nl:(e + 1) * nl]
        B[e] = Ball[:, k - p:k + 1]
        D[e] = Dall[:, k - p:k + 1]
        # every other function must vanish on this element
        rest = np.delete(Ball, np.arange(k - p, k + 1), axis=1)
        assert np.all(rest == 0.0)
    return kv, first, B, D, wg * 0.5 * h


def assemble(p, ne, hyper_every=0, alpha=0.0, beta=0.0, c_elem=None):
    """Return (K, M, C) as CSR matrices on the Dirichlet dofs.

    Each element's local matrices are computed by the 2-D tensor Gauss rule
    directly from the 2-D basis values, then summed into the global matrices.
    """
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n_all = n_functions(kv, p)
    n1 = n_all - 2
    nl = p + 1
    # 2-D values at the (p+1)^2 points: index q2 = (qy, qx), l2 = (ly, lx)
    W2 = np.outer(w, w).reshape(-1)                     # [qy*nl+qx]
    rows_k, cols_k, vk, vm, vc = [], [], [], [], []
    lx = np.arange(nl)
    for ey in range(ne):
        By, Dy = B[ey], D[ey]                            # [qy, ly]
        # Phi[ex, qy, qx, ly, lx]
        Phi = np.einsum("yb,xqa->xyqba", By, B)          # x=ex, y=qy, q=qx, b=ly, a=lx
        Gx = np.einsum("yb,xqa->xyqba", By, D)           # d/dx
        Gy = np.einsum("yb,xqa->xyqba", Dy, B)           # d/dy
        Phi = Phi.reshape(ne, nl * nl, nl * nl)
        Gx = Gx.reshape(ne, nl * nl, nl * nl)
        Gy = Gy.reshape(ne, nl * nl, nl * nl)
        Me = np.einsum("q,eqa,eqb->eab", W2, Phi, Phi)
        Ke = np.einsum("q,eqa,eqb->eab", W2, Gx, Gx) + np.einsum("q,eqa,eqb->eab", W2, Gy, Gy)
        Ce = alpha * Me + beta * Ke
        if c_elem is not None:
            Ce = Ce + np.asarray(c_elem)[ey][:, None, None] * Me
        # global 1-D indices of the local functions, then Dirichlet dof numbers
        gy = first[ey] + np.arange(nl)                   # [ly]
        gx = first[:, None] + lx[None, :]                # [ex, lx]
        okx = (gx >= 1) & (gx <= n1)
        oky = (gy >= 1) & (gy <= n1)
        dof = (gy[None, :, None] - 1) * n1 + (gx[:, None, :] - 1)   # [ex, ly, lx]
        ok = (oky[None, :, None] & okx[:, None, :]).reshape(ne, -1)
        dof = dof.reshape(ne, -1)
        R = np.broadcast_to(dof[:, :, None], Me.shape)
        Cc = np.broadcast_to(dof[:, None, :], Me.shape)
        mask = ok[:, :, None] & ok[:, None, :]
        rows_k.append(R[mask]); cols_k.append(Cc[mask])
        vk.append(Ke[mask]); vm.append(Me[mask]); vc.append(Ce[mask])
    r = np.concatenate(rows_k); c = np.concatenate(cols_k)
    N = n1 * n1
    K = sp.csr_matrix((np.concatenate(vk), (r, c)), shape=(N, N))
    M = sp.csr_matrix((np.concatenate(vm), (r, c)), shape=(N, N))
    C = sp.csr_matrix((np.concatenate(vc), (r, c)), shape=(N, N))
    for A in (K, M, C):
        A.sum_duplicates()
        A.sort_indices()
    return K, M, C


def assemble_1d(p, ne, hyper_every=0):
    """1-D stiffness and mass matrices (dense) on the Dirichlet functions:
    k_ij = int B_i' B_j', m_ij = int B_i B_j over [0, 1]."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n1 = n_functions(kv, p) - 2
    K1 = np.zeros((n1 + 2, n1 + 2))
    M1 = np.zeros((n1 + 2, n1 + 2))
    for e in range(ne):
        g = first[e] + np.arange(p + 1)
        M1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, B[e], B[e])
        K1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, D[e], D[e])
    return K1[1:-1, 1:-1], M1[1:-1, 1:-1]


def assemble_full_nodirichlet(p, ne, hyper_every=0):
    """K and M over *all* functions (no boundary elimination), dense; for the
    partition-of-unity checks on small meshes."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n = n_functions(kv, p)
    K1 = np.zeros((n, n)); M1 = np.zeros((n, n))
    for e in range(ne):
        g = first[e] + np.arange(p + 1)
        M1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, B[e], B[e])
        K1[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, D[e], D[e])
    return K1, M1


def entry(p, ne, hyper_every, a, b, alpha=0.0, beta=0.0, c_elem=None):
    """(K_ab, M_ab, C_ab) for one pair of Dirichlet dofs, by summing the 2-D
    Gauss rule over the elements where both functions are nonzero.  Used to
    check sampled entries of matrices too large for the full oracle."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n1 = n_functions(kv, p) - 2
    ax, ay = a % n1 + 1, a // n1 + 1
    bx, by = b % n1 + 1, b // n1 + 1
    k = m = c = 0.0
    for ey in range(ne):
        ly_a, ly_b = ay - first[ey], by - first[ey]
        if not (0 <= ly_a <= p and 0 <= ly_b <= p):
            continue
        for ex in range(ne):
            lx_a, lx_b = ax - first[ex], bx - first[ex]
            if not (0 <= lx_a <= p and 0 <= lx_b <= p):
                continue
            me = ke = 0.0
            for qy in range(p + 1):
                for qx in range(p + 1):
                    ww = w[qx] * w[qy]
                    va = B[ex, qx, lx_a] * B[ey, qy, ly_a]
                    vb = B[ex, qx, lx_b] * B[ey, qy, ly_b]
                    gxa = D[ex, qx, lx_a] * B[ey, qy, ly_a]
                    gya = B[ex, qx, lx_a] * D[ey, qy, ly_a]
                    gxb = D[ex, qx, lx_b] * B[ey, qy, ly_b]
                    gyb = B[ex, qx, lx_b] * D[ey, qy, ly_b]
                    me += ww * va * vb
                    ke += ww * (gxa * gxb + gya * gyb)
            m += me
            k += ke
            ce = alpha * me + beta * ke
            if c_elem is not None:
                ce += c_elem[ey, ex] * me
            c += ce
    return k, m, c


def element_mass_2d(p, ne, hyper_every, ex, ey):
    """(dofs, M_e) of one element restricted to Dirichlet dofs, for the adjoint."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n1 = n_functions(kv, p) - 2
    nl = p + 1
    dofs, vals = [], None
    W2 = np.outer(w, w)
    Phi = np.einsum("yb,xa->yxba", B[ey], B[ex]).reshape(nl * nl, nl * nl)
    Me = np.einsum("q,qa,qb->ab", W2.reshape(-1), Phi, Phi)
    for ly in range(nl):
        for lx in range(nl):
            gx, gy = first[ex] + lx, first[ey] + ly
            dofs.append((gy - 1) * n1 + (gx - 1) if (1 <= gx <= n1 and 1 <= gy <= n1) else -1)
    return np.array(dofs), Me


def q_matrix(K, M, C, sigma):
    """Q(sigma) = sigma^2 M + sigma C + K (Sec. 4.2), SPD for sigma > 0."""
    return (sigma * sigma) * M + sigma * C + K
