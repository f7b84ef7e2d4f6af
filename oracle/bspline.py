"""Univariate B-splines on open knot vectors (Sec. 3.1).

Oracle module: test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def knot_vector(p: int, ne: int, hyper_every: int = 0, mult: int | None = None) -> np.ndarray:
    """Open knot vector on [0, 1] with `ne` uniform elements (eq. KnotsX).

    The first and last knots are repeated p+1 times.  Interior knots k/ne have
    multiplicity 1 (maximum continuity C^{p-1}, Sec. 3.2).  rIGA (Sec. 3.3)
    raises the multiplicity at the hyperplanes, here every `hyper_every`
    elements, to `mult` (default p, i.e. C^0 separators); continuity at a knot
    of multiplicity r is C^{p-r}.
    """
    if mult is None:
        mult = p
    knots = [0.0] * (p + 1)
    for k in range(1, ne):
        r = mult if (hyper_every and k % hyper_every == 0) else 1
        knots += [k / ne] * r
    knots += [1.0] * (p + 1)
    return np.asarray(knots, dtype=np.float64)


def n_functions(knots: np.ndarray, p: int) -> int:
    return len(knots) - p - 1


def basis(knots: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """All degree-p B-splines at points x by the Cox--de Boor recursion.

    Degree 0 is the indicator of the half-open span [t_i, t_{i+1})
    (eq. BasisFunBi0); degree k combines two degree-(k-1) functions with the
    linear weights of eq. BasisFunBip.  A term whose denominator vanishes
    (repeated knots) is dropped, which is the 0/0 := 0 convention.
    Returns an array of shape (len(x), n_functions).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = knots
    nspan = len(t) - 1
    N = np.zeros((len(x), nspan))
    for i in range(nspan):
        N[:, i] = ((t[i] <= x) & (x < t[i + 1])).astype(np.float64)
    for k in range(1, p + 1):
        Nk = np.zeros((len(x), nspan - k))
        for i in range(nspan - k):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                Nk[:, i] += (x - t[i]) / d1 * N[:, i]
            if d2 > 0:
                Nk[:, i] += (t[i + k + 1] - x) / d2 * N[:, i + 1]
        N = Nk
    return N


def basis_deriv(knots: np.ndarray, p: int, x: np.ndarray) -> np.ndarray:
    """First derivatives of all degree-p B-splines at x.

    Differentiating eq. BasisFunBip gives
        B_i^p' = p/(t_{i+p}-t_i) B_i^{p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1}^{p-1},
    with a term dropped when its knot difference is zero.
    """
    t = knots
    Nm = basis(t, p - 1, x)  # degree p-1 on the same knots: one more function
    n = n_functions(t, p)
    D = np.zeros((Nm.shape[0], n))
    for i in range(n):
        d1 = t[i + p] - t[i]
        d2 = t[i + p + 1] - t[i + 1]
        if d1 > 0:
            D[:, i] += p / d1 * Nm[:, i]
        if d2 > 0:
            D[:, i] -= p / d2 * Nm[:, i + 1]
    return D


def gauss_legendre(npts: int):
    """Gauss--Legendre nodes and weights on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(npts)


def element_breaks(ne: int) -> np.ndarray:
    """Element boundaries of the uniform mesh on [0, 1]."""
    return np.arange(ne + 1, dtype=np.float64) / ne
