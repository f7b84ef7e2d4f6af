"""Pins of the divergence-conforming oracle (oracle/hdiv.py) against facts it
does not compute itself: the rotation to the curl-conforming space (div v =
rot u and |v| = |u| for v = (u_y, -u_x), relating two independent element
assemblies), the printed sizes of fig. MatPatterns (the spaces are rotations
of each other, Sec. 3.2), the wall integral of a constant normal component,
and the stability and Hamiltonian structure of the vibroacoustic QEP; planted
mistakes must fail them."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cshift
from oracle import eigen as oeig
from oracle import hcurl, hdiv

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig_matpatterns.json")
ALL = hdiv.LEFT | hdiv.RIGHT | hdiv.BOTTOM | hdiv.TOP


@pytest.mark.parametrize("p,ne,s", [(2, 6, 3), (3, 8, 4), (3, 8, 0), (4, 8, 4)])
def test_rotation_of_the_curl_conforming_space(p, ne, s):
    K, M, C = hdiv.assemble_hdiv(p, ne, s, 0)
    Kc, Mc, _ = hcurl.assemble_hcurl(p, ne, s, True)
    P = hdiv.rotation(p, ne, s)
    scale = abs(K).max()
    assert abs(K - P @ Kc @ P.T).max() <= 1e-14 * scale
    assert abs(M - P @ Mc @ P.T).max() <= 1e-14 * abs(M).max()
    assert C.nnz == K.nnz and abs(C).max() == 0.0
    # planted: without the sign of the rotated component the coupling flips
    Pn = abs(P)
    assert abs(K - Pn @ Kc @ Pn.T).max() > 1e-3 * scale


def test_fig_matpatterns_sizes():
    """64x64, p=4, no wall condition: N and nnz of the divergence-conforming
    IGA and rIGA (16x16 macroelements) spaces equal the printed ones."""
    g = json.load(open(GOLD))
    for s, key in ((0, "iga"), (g["macro"], "riga")):
        kvA, kvB, nA, (x0, x1), (y0, y1) = hdiv.spaces(g["p"], g["ne"], s, ALL)
        n = (x1 - x0) * nA + nA * (y1 - y0)
        assert n == g[key]["N"]
    K, _, _ = hdiv.assemble_hdiv(g["p"], 16, 4, ALL)
    Kc, _, _ = hcurl.assemble_hcurl(g["p"], 16, 4, False)
    assert K.shape == Kc.shape and K.nnz == Kc.nnz


@pytest.mark.parametrize("wall", [hdiv.LEFT, hdiv.RIGHT, hdiv.BOTTOM, hdiv.TOP])
def test_wall_integral_of_a_constant_normal_component(wall):
    """A field whose normal component is 1 on the absorbing wall (the end
    B function times the partition of unity of A) gives int_wall 1 = 1; the
    interior normal functions give 0."""
    p, ne, s = 3, 8, 4
    K0, _, _ = hdiv.assemble_hdiv(p, ne, s, wall, 0.0, 0.0)
    K1, _, C = hdiv.assemble_hdiv(p, ne, s, wall, 2.0, 1.0)
    kvA, kvB, nA, (x0, x1), (y0, y1) = hdiv.spaces(p, ne, s, wall)
    nBx, nBy = x1 - x0, y1 - y0
    base1 = nBx * nA
    N = K0.shape[0]
    c = np.zeros(N)
    if wall in (hdiv.LEFT, hdiv.RIGHT):
        i = 0 if wall == hdiv.LEFT else nBx - 1
        for j in range(nA):
            c[j * nBx + i] = 1.0
    else:
        j = 0 if wall == hdiv.BOTTOM else nBy - 1
        c[base1 + j * nA: base1 + (j + 1) * nA] = 1.0
    assert abs(c @ C @ c - 1.0) <= 1e-13
    assert abs(c @ (K1 - K0) @ c - 2.0) <= 1e-13
    interior = np.zeros(N)
    interior[:base1] = 1.0 if wall in (hdiv.BOTTOM, hdiv.TOP) else 0.0
    assert abs(interior @ C @ interior) <= 1e-15
    # planted: the opposite end function is not on this wall
    d = np.zeros(N)
    if wall in (hdiv.LEFT, hdiv.RIGHT):
        i = nBx - 1 if wall == hdiv.LEFT else 0
        for j in range(nA):
            d[j * nBx + i] = 1.0
    else:
        j = nBy - 1 if wall == hdiv.BOTTOM else 0
        d[base1 + j * nA: base1 + (j + 1) * nA] = 1.0
    assert abs(d @ C @ d - 1.0) > 0.5


def test_vibroacoustic_qep_is_stable_and_real():
    """K, C semidefinite and M definite (eq. HdivQuadEig): every eigenvalue
    has Re lam <= 0 and the spectrum is closed under conjugation; without
    damping it is purely imaginary; ARPACK's real-part mode at a complex
    target agrees with dense QZ.  (The divergence-free fields with a zero
    normal trace on the absorbing wall give lam = 0 twice, a Jordan pair that
    QZ resolves only to sqrt(eps): that cluster is left out of the sign
    checks.)"""
    p, ne, s = 2, 6, 3
    K, M, C = hdiv.assemble_hdiv(p, ne, s, hdiv.TOP, 0.5, 0.8)
    lam = oeig.dense_qep(K, C, M)[0]
    lam = lam[np.isfinite(lam)]
    scale = np.abs(lam).max()
    lam = lam[np.abs(lam) > 1e-5 * scale]
    assert lam.real.max() <= 1e-9 * scale
    for x in lam[np.abs(lam.imag) > 1e-8 * scale][:20]:
        assert np.min(np.abs(lam - np.conj(x))) <= 1e-8 * scale
    assert np.linalg.eigvalsh(M.toarray()).min() > 0
    assert np.linalg.eigvalsh(C.toarray()).min() >= -1e-14
    sigma = 0.5 + 6.0j
    ref = cshift.select(lam, sigma, 10)
    ar = cshift.real_part_arpack(K, C, M, sigma, 10)
    assert np.abs(ar - ref).max() <= 1e-9 * np.abs(ref).max()
    K0, M0, C0 = hdiv.assemble_hdiv(p, ne, s, hdiv.TOP, 0.5, 0.0)
    lam0 = oeig.dense_qep(K0, C0, M0)[0]
    lam0 = lam0[np.isfinite(lam0)]
    lam0 = lam0[np.abs(lam0) > 1e-5 * np.abs(lam0).max()]
    assert np.abs(lam0.real).max() <= 1e-8 * np.abs(lam0).max()
    # planted: the damping's sign reversed makes some modes grow
    lamn = oeig.dense_qep(K, -C, M)[0]
    assert lamn[np.isfinite(lamn)].real.max() > 1e-3
