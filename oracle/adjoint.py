"""Sensitivity of QEP eigenvalues to a per-element damping field.

Oracle module: test infrastructure only.

For C = C0 + sum_e c_e M_e the pencil Q(lam) = K + lam C + lam^2 M is
complex-symmetric (real symmetric K, C, M), so the left eigenvector of a
simple eigenvalue is the complex conjugate of the right one, u.  Differentiating
u^T Q(lam) u = 0 (unconjugated transpose) with respect to c_e gives
    d lam / d c_e = - lam u^T M_e u / u^T (2 lam M + C) u.
For L = sum_k Re lam_k:  dL/dc_e = sum_k Re(d lam_k / d c_e).
"""
from __future__ import annotations

import numpy as np

from .assemble import _element_tables
from .bspline import n_functions


def element_quadratic_forms(p, ne, hyper_every, U):
    """q[k, ey, ex] = u_k^T M_e u_k (unconjugated) for the columns u_k of U."""
    kv, first, B, D, w = _element_tables(p, ne, hyper_every)
    n1 = n_functions(kv, p) - 2
    nl = p + 1
    U = np.asarray(U)
    if U.ndim == 1:
        U = U[:, None]
    nvec = U.shape[1]
    # local 1-D mass blocks: mloc[e, a, b] = int_e B_a B_b
    mloc = np.einsum("q,eqa,eqb->eab", w, B, B)
    out = np.zeros((nvec, ne, ne), dtype=U.dtype)
    for ey in range(ne):
        for ex in range(ne):
            gx = first[ex] + np.arange(nl)
            gy = first[ey] + np.arange(nl)
            okx = (gx >= 1) & (gx <= n1)
            oky = (gy >= 1) & (gy <= n1)
            # element mass on the tensor local basis: M_e = my (x) mx
            Me = np.kron(mloc[ey][np.ix_(oky, oky)], mloc[ex][np.ix_(okx, okx)])
            dofs = ((gy[oky] - 1)[:, None] * n1 + (gx[okx] - 1)[None, :]).reshape(-1)
            ue = U[dofs, :]
            out[:, ey, ex] = np.einsum("ak,ab,bk->k", ue, Me, ue)
    return out


def dlam_dc(p, ne, hyper_every, M, C, lam, U):
    """d lam_k / d c_e for each eigenpair (lam_k, u_k): array (nev, ne, ne)."""
    lam = np.atleast_1d(lam)
    U = np.asarray(U).reshape(M.shape[0], -1)
    q = element_quadratic_forms(p, ne, hyper_every, U)
    out = np.zeros_like(q, dtype=np.complex128)
    for k in range(len(lam)):
        u = U[:, k]
        den = u @ (2 * lam[k] * (M @ u) + C @ u)
        out[k] = -lam[k] * q[k] / den
    return out


def grad_sum_re(p, ne, hyper_every, M, C, lam, U):
    """dL/dc_e for L = sum_k Re(lam_k), shape (ne, ne) indexed [ey, ex]."""
    return np.real(dlam_dc(p, ne, hyper_every, M, C, lam, U)).sum(axis=0)
