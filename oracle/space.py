"""Dimensions and sparsity of IGA / rIGA spaces (Sec. 3.2, 3.3, fig. MatPatterns).

Oracle module: test infrastructure only.

A B-spline B_i^p on knots t is supported on [t_i, t_{i+p+1}].  Two basis
functions couple in a Galerkin matrix exactly when their supports overlap on
a set of positive length; a tensor-product pair couples when both of its
1-D factors do.
"""
from __future__ import annotations

import numpy as np

from .bspline import knot_vector, n_functions


def supports(knots: np.ndarray, p: int) -> np.ndarray:
    """(n, 2) array of [start, end] of every function's support."""
    n = n_functions(knots, p)
    return np.array([[knots[i], knots[i + p + 1]] for i in range(n)])


def overlap_pairs(sa: np.ndarray, sb: np.ndarray) -> int:
    """Number of ordered pairs (a in A, b in B) whose supports overlap."""
    lo = np.maximum(sa[:, None, 0], sb[None, :, 0])
    hi = np.minimum(sa[:, None, 1], sb[None, :, 1])
    return int(np.count_nonzero(hi > lo))


def n1d_dirichlet(p: int, ne: int, hyper_every: int = 0) -> int:
    """1-D dimension of the scalar space after removing the two end functions
    (the only ones that do not vanish on the boundary of an open knot vector)."""
    return n_functions(knot_vector(p, ne, hyper_every), p) - 2


def scalar_counts(p: int, ne: int, hyper_every: int = 0):
    """(N, nnz) of the scalar H^1 Dirichlet space S^{p,p} with C^0 hyperplanes."""
    kv = knot_vector(p, ne, hyper_every)
    s = supports(kv, p)[1:-1]
    n1 = len(s)
    ov = overlap_pairs(s, s)
    return n1 * n1, ov * ov


def hcurl_counts(p: int, ne: int, macro: int = 0):
    """(N, nnz) of the H(curl) space S^{p-1,p} x S^{p,p-1} of Sec. 3.2.

    Maximum continuity is k = p-1 in the degree-p direction and k-1 in the
    degree-(p-1) direction.  rIGA (Sec. 3.3) lowers both by k-1 = p-2 at the
    hyperplanes, i.e. to C^1 and C^0 respectively; either way the hyperplane
    knot multiplicity is p-1.  No boundary functions are removed: the counts
    are those of the assembled system matrix of fig. MatPatterns.
    """
    ku = knot_vector(p - 1, ne, macro, mult=p - 1)
    kv = knot_vector(p, ne, macro, mult=p - 1)
    su, sv = supports(ku, p - 1), supports(kv, p)
    nu, nv = len(su), len(sv)
    n = 2 * nu * nv
    nnz = 2 * overlap_pairs(su, su) * overlap_pairs(sv, sv) + 2 * overlap_pairs(su, sv) ** 2
    return n, nnz
