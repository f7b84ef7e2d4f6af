"""The gyroscopic damped-wave QEP: damping with a skew-symmetric part.

Oracle module: test infrastructure only.

The model-problem remark of Sec. 2.1 (after eq. HcurlQuadEig) treats a
damping matrix that is skew-Hermitian, C = -C^T: a gyroscopic eigensystem
whose spectrum is Hamiltonian (symmetric with respect to the imaginary axis).
Here the skew part is real: the convection-type form of a constant vector
g = (gx, gy),
    G_ab = int_Omega B_a (g . grad B_b),
which is skew-symmetric on the Dirichlet space (integration by parts, the
boundary term vanishes), and
    C = alpha M + beta K + G,     Q(lam) = K + lam C + lam^2 M.
With alpha = beta = 0 every eigenvalue is purely imaginary (K, M SPD, G skew).

Routes (independent of each other and of the HIP library):
  * assemble_gyro     -- K, M, C with G integrated element by element with the
                         2-D tensor Gauss rule from the 2-D basis values;
  * assemble_1d_skew  -- the 1-D matrix s_ij = int B_i B_j' (Dirichlet
                         functions, or all functions for the pins);
  * gyro_closed       -- gy = 0: on the identity geometry
                         K = M1 (x) K1 + K1 (x) M1, M = M1 (x) M1 and
                         G = gx M1 (x) S1 (x fastest), so every 1-D y-mode
                         (mu_j, phi_j) of K1 phi = mu M1 phi reduces the QEP to
                         the 1-D QEP in x
                           (K1 + mu_j M1) + lam (alpha M1 + beta (K1 + mu_j M1) + gx S1) + lam^2 M1,
                         and the 2-D spectrum is the union over j; each 1-D
                         QEP is solved for its eigenvalues nearest sigma by
                         sparse shift-and-invert (eigen.shift_invert);
  * eigen.dense_qep   -- QZ on the full companion pencil (tiny meshes).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import _element_tables, assemble, assemble_1d
from .bspline import knot_vector, n_functions
from .eigen import canonical_order, mu_1d, shift_invert


def assemble_1d_skew(p, ne, hyper_every=0, dirichlet=True):
    """s_ij = int_0^1 B_i(x) B_j'(x) dx (dense), on the Dirichlet functions or
    (dirichlet=False) on all of them."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n = n_functions(kv, p)
    S = np.zeros((n, n))
    for e in range(ne):
        g = first[e] + np.arange(p + 1)
        S[np.ix_(g, g)] += np.einsum("q,qa,qb->ab", w, B[e], D[e])
    return S[1:-1, 1:-1] if dirichlet else S


def greville(p, ne, hyper_every=0):
    """Greville abscissae (t_{j+1} + ... + t_{j+p}) / p of every function:
    sum_j g_j B_j(x) = x on [0, 1] for p >= 1."""
    kv = knot_vector(p, ne, hyper_every)
    n = n_functions(kv, p)
    return np.array([kv[j + 1:j + p + 1].mean() for j in range(n)])


def assemble_gyro(p, ne, hyper_every=0, alpha=0.0, beta=0.0, gx=0.0, gy=0.0):
    """(K, M, C) in CSR on the Dirichlet dofs with C = alpha M + beta K + G,
    G_ab = int B_a (gx dB_b/dx + gy dB_b/dy) by the 2-D tensor Gauss rule on
    every element (row a, column b)."""
    K, M, _ = assemble(p, ne, hyper_every)
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n1 = n_functions(kv, p) - 2
    nl = p + 1
    W2 = np.outer(w, w).reshape(-1)
    lx = np.arange(nl)
    rows, cols, vals = [], [], []
    for ey in range(ne):
        By, Dy = B[ey], D[ey]
        Phi = np.einsum("yb,xqa->xyqba", By, B).reshape(ne, nl * nl, nl * nl)
        Gx = np.einsum("yb,xqa->xyqba", By, D).reshape(ne, nl * nl, nl * nl)
        Gy = np.einsum("yb,xqa->xyqba", Dy, B).reshape(ne, nl * nl, nl * nl)
        Ge = gx * np.einsum("q,eqa,eqb->eab", W2, Phi, Gx) + gy * np.einsum("q,eqa,eqb->eab", W2, Phi, Gy)
        gyi = first[ey] + np.arange(nl)
        gxi = first[:, None] + lx[None, :]
        okx = (gxi >= 1) & (gxi <= n1)
        oky = (gyi >= 1) & (gyi <= n1)
        dof = ((gyi[None, :, None] - 1) * n1 + (gxi[:, None, :] - 1)).reshape(ne, -1)
        ok = (oky[None, :, None] & okx[:, None, :]).reshape(ne, -1)
        R = np.broadcast_to(dof[:, :, None], Ge.shape)
        Cc = np.broadcast_to(dof[:, None, :], Ge.shape)
        mask = ok[:, :, None] & ok[:, None, :]
        rows.append(R[mask]); cols.append(Cc[mask]); vals.append(Ge[mask])
    N = n1 * n1
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    G.sum_duplicates()
    # C on the stored pattern of K and M (G's entries lie where two supports
    # meet; a sparse sum would drop entries that happen to be zero)
    Cfull = (alpha * M + beta * K + G).tocsr()
    C = K.copy()
    r, c = K.nonzero()
    C.data = np.asarray(Cfull[r, c]).ravel()
    return K, M, C


def _modulus_lower_bound(mu, nu_min, nu_max, alpha, beta, gx):
    """A lower bound on |lam| over the eigenvalues of the 1-D QEP of a y-mode
    mu.  For an eigenpair (lam, w), with m = w^H M1 w, t = w^H K1 w / m in
    [nu_min, nu_max] (the 1-D Rayleigh quotient range) and c the damping form
    w^H (alpha M1 + beta (K1 + mu M1) + gx S1) w, lam is a root of
    m lam^2 + c lam + (t + mu) m = 0, where |c| / m <= alpha + beta (t + mu)
    + |gx| sqrt(t) (Cauchy--Schwarz: |w^H S1 w| <= ||w||_M1 ||w'||_M1).  The
    product of the roots is t + mu and their sum is bounded by |c| / m, so
    the smaller modulus is at least (-b + sqrt(b^2 + 4 (t + mu))) / 2 with b
    that bound.  Minimised over t on a fine logarithmic grid and lowered by
    10 % as a margin for the grid."""
    t = np.geomspace(nu_min, nu_max, 4000)
    b = alpha + beta * (t + mu) + abs(gx) * np.sqrt(t)
    f = (-b + np.sqrt(b * b + 4.0 * (t + mu))) * 0.5
    return 0.9 * float(f.min())


def gyro_closed(p, ne, hyper_every, alpha, beta, gx, sigma, nev, k0=8):
    """The nev eigenvalues nearest sigma (> 0) of the QEP with
    C = alpha M + beta K + gx M1 (x) S1 (gy = 0), in canonical order, from the
    1-D QEPs of the y-modes, taken in increasing mu_j.  A mode is searched
    until the k eigenvalues nearest sigma it returns reach the current nev-th
    distance R (k doubled; its whole spectrum densely when that is smaller);
    modes stop once the lower bound on |lam| of the next mode exceeds
    sigma + R, and every searched mode is searched again while its radius is
    below the final R."""
    from .eigen import dense_qep
    K1, M1 = assemble_1d(p, ne, hyper_every)
    S1 = assemble_1d_skew(p, ne, hyper_every)
    n = K1.shape[0]
    kmax = 2 * n - 3
    mus = mu_1d(p, ne, hyper_every)
    nu_min, nu_max = float(mus[0]), float(mus[-1])
    K1s, M1s, S1s = sp.csr_matrix(K1), sp.csr_matrix(M1), sp.csr_matrix(S1)
    v0 = np.ones(2 * n)
    found, radius, ks = {}, {}, {}

    def search(j, k):
        mu = mus[j]
        Kj = (K1s + mu * M1s).tocsr()
        Cj = (alpha * M1s + beta * Kj + gx * S1s).tocsr()
        if k < kmax and 2 * n > 60:
            try:
                lam = shift_invert(Kj, Cj, M1s, sigma, k, extra=0, v0=v0)
                found[j], radius[j], ks[j] = lam, float(np.max(np.abs(lam - sigma))), k
                return
            except Exception:   # ARPACK without convergence: the dense route
                pass
        found[j], radius[j], ks[j] = dense_qep(Kj, Cj, M1s)[0], np.inf, kmax

    def current_R():
        allv = np.concatenate([found[j] for j in found]) if found else np.zeros(0)
        if len(allv) < nev:
            return np.inf
        return float(np.sort(np.abs(allv - sigma))[nev - 1])

    for j in range(len(mus)):
        if _modulus_lower_bound(mus[j], nu_min, nu_max, alpha, beta, gx) > sigma + current_R():
            break
        search(j, min(k0, kmax))
        while radius[j] < current_R() and ks[j] < kmax:
            search(j, min(2 * ks[j], kmax))
    while True:
        R = current_R()
        todo = [j for j in found if radius[j] < R and ks[j] < kmax]
        if not todo:
            break
        for j in todo:
            search(j, min(2 * ks[j], kmax))
    cand = np.concatenate([found[j] for j in found])
    return cand[canonical_order(cand, sigma)[:nev]]
