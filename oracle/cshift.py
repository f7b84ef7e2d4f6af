"""A complex target shift for the real QEP (K + lam C + lam^2 M) u = 0
(Sec. 4.1.1, shift-and-invert with a complex shift; the target of Alg. 2
placed inside the complex spectrum region of interest).

Oracle module: test infrastructure only.

With real K, C, M the spectrum is closed under conjugation, and the real part
of the shift-and-invert operator,
    Re S(sigma) = (S(sigma) + S(conj sigma)) / 2,  S(s) = (A - s B)^{-1} B
(A, B the companion pencil of eq. Linearization), is a real operator whose
eigenvectors are the pencil's, with the values
    psi(lam) = (1/(lam - sigma) + 1/(lam - conj sigma)) / 2
(the real-part operator of Parlett and Saad, "Complex shift and invert
strategies for real matrices", 1987; ARPACK's mode 3 with a complex shift).
The eigenvalues such a solver returns first are those of largest |psi|: near
sigma or near conj sigma, in conjugate pairs.  This module defines that set:

  * psi, psi_order, select  -- the transform and the ordering by decreasing
                               |psi| (ties, e.g. conjugate pairs, by Im
                               descending, then Re ascending);
  * rayleigh_cshift         -- Rayleigh damping on the scalar space: every
                               eigenvalue from the 1-D closed form (all mode
                               pairs), then the selection;
  * maxwell_cshift          -- the same on the curl-conforming space with the
                               perfect conductor: the Maxwell values (sums of
                               1-D values) and the gradient null space, whose
                               modes give lam = 0 and lam = -alpha;
  * real_part_arpack        -- ARPACK on Re S(sigma) through SciPy (a second,
                               independent route for small meshes).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .eigen import mu_1d, quad_roots
from . import hcurl


def psi(lam, sigma: complex):
    """(1/(lam - sigma) + 1/(lam - conj sigma)) / 2, elementwise."""
    lam = np.asarray(lam, dtype=complex)
    return 0.5 * (1.0 / (lam - sigma) + 1.0 / (lam - np.conj(sigma)))


def psi_order(lam, sigma: complex, rel: float = 1e-9) -> np.ndarray:
    """Indices sorting lam by decreasing |psi|; values whose |psi| agree to
    `rel` (relative) form a cluster ordered by Im descending, then Re
    ascending."""
    lam = np.asarray(lam, dtype=complex)
    g = np.abs(psi(lam, sigma))
    idx = np.argsort(-g, kind="stable")
    out = []
    i = 0
    while i < len(idx):
        j = i + 1
        g0 = g[idx[i]]
        while j < len(idx) and g0 - g[idx[j]] <= rel * g0:
            j += 1
        out.extend(sorted(idx[i:j], key=lambda k: (-lam[k].imag, lam[k].real)))
        i = j
    return np.asarray(out, dtype=np.int64)


def select(lam, sigma: complex, nev: int) -> np.ndarray:
    lam = np.asarray(lam, dtype=complex)
    return lam[psi_order(lam, sigma)[:nev]]


def _roots(mus, alpha, beta):
    """Both roots of lam^2 + (alpha + beta mu) lam + mu = 0 for every mu."""
    mus = np.asarray(mus, dtype=float)
    r1, r2 = quad_roots(1.0, alpha + beta * mus, mus)
    return np.concatenate([np.asarray(r1, dtype=complex), np.asarray(r2, dtype=complex)])


def rayleigh_cshift(p, ne, hyper_every, alpha, beta, sigma, nev):
    """The nev eigenvalues of largest |psi| for C = alpha M + beta K on the
    scalar Dirichlet space: mu_ij = mu_i + mu_j over every pair of 1-D values
    (K = K1 (x) M1 + M1 (x) K1, M = M1 (x) M1), both roots of each."""
    mu1 = mu_1d(p, ne, hyper_every)
    mus = (mu1[:, None] + mu1[None, :]).reshape(-1)
    return select(_roots(mus, alpha, beta), sigma, nev)


def maxwell_cshift(p, ne, hyper_every, alpha, beta, sigma, nev):
    """The nev eigenvalues of largest |psi| for C = alpha M + beta K on the
    curl-conforming space with the perfect conductor: every nonzero Maxwell
    value, plus the null space (mu = 0, multiplicity null_dimension), whose
    roots are 0 and -alpha."""
    nz = hcurl.maxwell_closed(p, ne, hyper_every, True, 1e-300, np.inf)
    null = hcurl.null_dimension(p, ne, hyper_every, True)
    lam = np.concatenate([_roots(nz, alpha, beta), np.zeros(null, dtype=complex),
                          np.full(null, -alpha, dtype=complex)])
    return select(lam, sigma, nev)


def real_part_arpack(K, C, M, sigma, nev):
    """ARPACK (SciPy, OPpart='r') on Re S(sigma) for the companion pencil
    A = [[0, I], [-K, -C]], B = diag(I, M): its eigenvalues are recovered
    from the eigenvectors, in psi order."""
    K = sp.csr_matrix(K); C = sp.csr_matrix(C); M = sp.csr_matrix(M)
    n = K.shape[0]
    Z = sp.csr_matrix((n, n)); I = sp.identity(n, format="csr")
    A = sp.bmat([[Z, I], [-K, -C]]).tocsc()
    B = sp.bmat([[I, Z], [Z, M]]).tocsc()
    w, _ = spla.eigs(A, k=nev, M=B, sigma=sigma, OPpart="r", which="LM", tol=1e-13)
    return w[psi_order(w, sigma)]
