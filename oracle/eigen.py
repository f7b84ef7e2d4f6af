"""Eigenvalues of the QEP (K + lam C + lam^2 M) u = 0 nearest a shift.

Oracle module: test infrastructure only.

Three independent routes to the same set:
  * dense_qep        -- QZ on the first companion pencil of eq. Linearization
                        (all 2N eigenvalues; tiny meshes only);
  * rayleigh_closed  -- Rayleigh damping C = alpha M + beta K: each eigenvector
                        of K phi = mu M phi gives lam^2 + (alpha + beta mu) lam
                        + mu = 0; on the identity geometry K = K1 (x) M1 +
                        M1 (x) K1 and M = M1 (x) M1, so mu_ij = mu_i + mu_j
                        from the 1-D pencil (any mesh size);
  * shift_invert     -- ARPACK on the operator S = L(s)^{-1} B applied through
                        eq. BlockOperatorVector with a sparse LU of Q(s).
Plus the scaled residual and the canonical ordering used to compare results.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import assemble_1d


# --- ordering -----------------------------------------------------------------

def canonical_order(lam: np.ndarray, sigma: float, rel: float = 1e-9) -> np.ndarray:
    """Indices sorting lam by distance to sigma; values whose distances agree
    to `rel` (relative) form a cluster, ordered by Im descending, then Re
    ascending."""
    lam = np.asarray(lam)
    d = np.abs(lam - sigma)
    idx = np.argsort(d, kind="stable")
    out = []
    i = 0
    while i < len(idx):
        j = i + 1
        d0 = d[idx[i]]
        while j < len(idx) and d[idx[j]] - d0 <= rel * max(d0, 1e-300):
            j += 1
        grp = idx[i:j]
        grp = sorted(grp, key=lambda k: (-lam[k].imag, lam[k].real))
        out.extend(grp)
        i = j
    return np.asarray(out, dtype=np.int64)


def nearest(lam: np.ndarray, sigma: float, nev: int) -> np.ndarray:
    lam = np.asarray(lam)
    return lam[canonical_order(lam, sigma)[:nev]]


# --- dense brute force ----------------------------------------------------------

def dense_qep(K, C, M):
    """All 2N eigenvalues (and upper-block eigenvectors) of the QEP from the
    companion pencil A - lam B with A = [[0, I], [-K, -C]], B = diag(I, M)
    (eq. Linearization), by LAPACK's QZ."""
    K = K.toarray() if sp.issparse(K) else np.asarray(K)
    C = C.toarray() if sp.issparse(C) else np.asarray(C)
    M = M.toarray() if sp.issparse(M) else np.asarray(M)
    n = K.shape[0]
    Z = np.zeros((n, n)); I = np.eye(n)
    A = np.block([[Z, I], [-K, -C]])
    B = np.block([[I, Z], [Z, M]])
    lam, V = sla.eig(A, B)
    return lam, V[:n, :]


# --- closed form for Rayleigh damping --------------------------------------------

def quad_roots(a: float, b: float, c: float):
    """Both roots of a lam^2 + b lam + c = 0 (complex)."""
    disc = np.lib.scimath.sqrt(b * b - 4 * a * c)
    return (-b + disc) / (2 * a), (-b - disc) / (2 * a)


def mu_1d(p, ne, hyper_every):
    """Eigenvalues of the 1-D pencil K1 phi = mu M1 phi, each polished by the
    Rayleigh quotient of its LAPACK eigenvector (the quotient's error is the
    square of the vector's, which removes the eps*mu_max absolute error of the
    direct solve on the small eigenvalues)."""
    K1, M1 = assemble_1d(p, ne, hyper_every)
    w, V = sla.eigh(K1, M1)
    rq = np.einsum("ik,ij,jk->k", V, K1, V) / np.einsum("ik,ij,jk->k", V, M1, V)
    return np.sort(rq)


def rayleigh_closed(p, ne, hyper_every, alpha, beta, sigma, nev, pad=8):
    """The nev QEP eigenvalues nearest sigma for C = alpha M + beta K, in
    canonical order, together with their generalised eigenvalues mu."""
    mu1 = mu_1d(p, ne, hyper_every)
    # distance to sigma grows with mu for both roots once the mode is
    # underdamped, so a modest number of the smallest mu suffices; take the
    # smallest nev+pad 1-D sums and all their roots.
    kk = min(len(mu1), nev + pad)
    mus = (mu1[:kk, None] + mu1[None, :kk]).reshape(-1)
    mus = np.sort(mus)[: 2 * (nev + pad)]
    lam, mu_of = [], []
    for mu in mus:
        r1, r2 = quad_roots(1.0, alpha + beta * mu, mu)
        lam += [complex(r1), complex(r2)]
        mu_of += [mu, mu]
    lam = np.asarray(lam); mu_of = np.asarray(mu_of)
    order = canonical_order(lam, sigma)[:nev]
    return lam[order], mu_of[order]


def generalized_mu(p, ne, hyper_every, count):
    """The `count` smallest eigenvalues of K u = mu M u in 2-D (with
    multiplicity), from the 1-D pencil."""
    mu1 = mu_1d(p, ne, hyper_every)
    kk = min(len(mu1), count + 1)
    mus = np.sort((mu1[:kk, None] + mu1[None, :kk]).reshape(-1))
    return mus[:count]


# --- sparse shift-and-invert -------------------------------------------------------

def shift_invert(K, C, M, sigma, nev, extra=6, tol=1e-13, v0=None, return_vectors=False):
    """Eigenvalues nearest sigma by ARPACK on S = L(sigma)^{-1} B, applied as in
    eq. BlockOperatorVector:
        r_u = -Q(sigma)^{-1} (sigma M v_u + C v_u + M v_l),  r_l = sigma r_u + v_u,
    with theta = 1/(lam - sigma) (eq. ShiftInvert)."""
    K = sp.csr_matrix(K); C = sp.csr_matrix(C); M = sp.csr_matrix(M)
    n = K.shape[0]
    Q = ((sigma * sigma) * M + sigma * C + K).tocsc()
    lu = spla.splu(Q)
    Ms = (sigma * M + C).tocsr()

    def op(v):
        v = np.asarray(v).reshape(-1)
        vu, vl = v[:n], v[n:]
        ru = -lu.solve(Ms @ vu + M @ vl)
        return np.concatenate([ru, sigma * ru + vu])

    S = spla.LinearOperator((2 * n, 2 * n), matvec=op, dtype=np.float64)
    k = min(nev + extra, 2 * n - 2)
    ncv = min(2 * n, max(2 * k + 1, 40))
    theta, V = spla.eigs(S, k=k, which="LM", tol=tol, v0=v0, ncv=ncv)
    lam = sigma + 1.0 / theta
    order = canonical_order(lam, sigma)[:nev]
    if return_vectors:
        return lam[order], V[:n, order]
    return lam[order]


# --- residual -------------------------------------------------------------------

def onenorm(A) -> float:
    A = sp.csr_matrix(A)
    return float(abs(A).sum(axis=0).max())


def residual(K, C, M, lam, u, norms=None) -> float:
    """Scaled backward error of an approximate eigenpair,
        eta = ||Q(lam) u||_2 / ((|lam|^2 ||M||_1 + |lam| ||C||_1 + ||K||_1) ||u||_2),
    the form of Tisseur's analysis cited in the scaling remark of Sec. 6.2.2
    (1-norms of the coefficient matrices)."""
    if norms is None:
        norms = (onenorm(K), onenorm(C), onenorm(M))
    nk, nc, nm = norms
    r = K @ u + lam * (C @ u) + lam * lam * (M @ u)
    return float(np.linalg.norm(r) / ((abs(lam) ** 2 * nm + abs(lam) * nc + nk) * np.linalg.norm(u)))
