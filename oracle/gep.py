"""The generalized eigenproblem K u = mu M u (no damping, C = 0) and its
inertia, for spectrum slicing.

Oracle module: test infrastructure only.

With C = 0 the QEP of eq. QuadEig reduces to the Hermitian definite pencil
(K, M): every eigenvalue mu is real and positive.  Sec. 4.1.4 (spectrum
slicing): for an LDL^T factorization K - s M = L D L^T, Sylvester's law of
inertia gives the number of eigenvalues below s as the number of negative
eigenvalues of D, so an interval [a, b) holds nu(b) - nu(a) eigenvalues
counted with multiplicity.

Routes (independent of each other and of the HIP library):
  * gep_closed       -- all mu in an interval from the Kronecker sums
                        mu_ij = mu_i + mu_j of the 1-D pencil (exact on the
                        identity geometry; any mesh size);
  * gep_dense        -- LAPACK's dense symmetric-definite solver (tiny meshes);
  * count_below      -- the closed-form count of eigenvalues below a shift;
  * inertia_dense    -- nu(K - s M) from LAPACK's symmetric indefinite
                        factorization (Bunch-Kaufman: D has 1x1 and 2x2
                        blocks, whose eigenvalues are counted).
Plus the scaled residual of an approximate pair.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .eigen import mu_1d, onenorm


def gep_closed(p, ne, hyper_every, a, b):
    """Every eigenvalue of K u = mu M u in [a, b), sorted, with multiplicity:
    the sums mu_i + mu_j (i, j over the 1-D spectrum, ordered pairs) that lie
    in the interval."""
    mu1 = mu_1d(p, ne, hyper_every)
    out = []
    for i in range(len(mu1)):
        if mu1[i] + mu1[0] >= b:
            break
        for j in range(len(mu1)):
            m = mu1[i] + mu1[j]
            if m >= b:
                break
            if m >= a:
                out.append(m)
    return np.sort(np.asarray(out, dtype=np.float64))


def count_below(p, ne, hyper_every, s):
    """The number of eigenvalues mu < s (with multiplicity), closed form."""
    return int(len(gep_closed(p, ne, hyper_every, -np.inf, s)))


def gep_dense(K, M):
    """All eigenvalues and M-orthonormal eigenvectors of K u = mu M u by
    LAPACK's dense symmetric-definite solver."""
    K = K.toarray() if sp.issparse(K) else np.asarray(K)
    M = M.toarray() if sp.issparse(M) else np.asarray(M)
    return sla.eigh(K, M)


def inertia_dense(K, M, s):
    """nu(K - s M): the negative eigenvalues of D in the symmetric indefinite
    factorization P (K - s M) P^T = L D L^T (Sylvester's law of inertia)."""
    K = K.toarray() if sp.issparse(K) else np.asarray(K)
    M = M.toarray() if sp.issparse(M) else np.asarray(M)
    _, D, _ = sla.ldl(K - s * M)
    return int(np.sum(np.linalg.eigvalsh(D) < 0))


def gep_residual(K, M, mu, u, norms=None):
    """||K u - mu M u||_2 / ((||K||_1 + |mu| ||M||_1) ||u||_2): the backward
    error form of the residual of the QEP with C = 0 at degree one."""
    if norms is None:
        norms = (onenorm(K), onenorm(M))
    nk, nm = norms
    r = K @ u - mu * (M @ u)
    return float(np.linalg.norm(r) / ((nk + abs(mu) * nm) * np.linalg.norm(u)))
