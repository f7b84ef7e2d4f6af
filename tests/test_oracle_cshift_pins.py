"""Pins of the complex-shift oracle (oracle/cshift.py) against facts it does
not compute itself: the transform's identities, LAPACK's dense QZ with the
selection written out, ARPACK's real-part operator (SciPy, OPpart='r') as an
independent route, and the closed forms on the scalar and curl-conforming
spaces; planted mistakes (nearest-to-sigma instead of largest |psi|, a
dropped null space) must fail them."""
import numpy as np
import pytest

from oracle import assemble as oasm
from oracle import cshift
from oracle import eigen as oeig
from oracle import hcurl


def test_psi_identities():
    """Real lam: psi = Re 1/(lam - sigma); psi(conj lam) = conj psi(lam);
    psi is the mean of the two shifted inverses, largest near sigma and conj
    sigma, and (lam - a) / ((lam - a)^2 + b^2) for sigma = a + ib."""
    sigma = 0.4 + 3.0j
    x = np.linspace(-5.0, 5.0, 11)
    assert np.allclose(cshift.psi(x, sigma), (1.0 / (x - sigma)).real, rtol=1e-15, atol=0)
    lam = np.array([-0.2 + 2.9j, 1.0 - 0.5j, -3.0 + 0.1j])
    assert np.allclose(cshift.psi(np.conj(lam), sigma), np.conj(cshift.psi(lam, sigma)), rtol=1e-15, atol=0)
    a, b = sigma.real, sigma.imag
    assert np.allclose(cshift.psi(lam, sigma), (lam - a) / ((lam - a) ** 2 + b * b), rtol=1e-14, atol=0)
    g = np.abs(cshift.psi(lam, sigma))
    assert g[0] > 4 * g[1] and g[0] > 4 * g[2]


@pytest.mark.parametrize("p,ne,s,sigma", [(2, 12, 4, 0.3 + 7.0j), (3, 10, 0, 0.0 + 5.0j), (2, 10, 5, 1.0 + 2.0j)])
def test_closed_form_and_arpack_match_dense_qz(p, ne, s, sigma):
    alpha, beta, nev = 0.05, 0.005, 12
    K, M, C = oasm.assemble(p, ne, s, alpha, beta)
    dense = oeig.dense_qep(K, C, M)[0]
    ref = cshift.select(dense, sigma, nev)
    lam = cshift.rayleigh_cshift(p, ne, s, alpha, beta, sigma, nev)
    scale = np.abs(ref).max()
    assert np.abs(lam - ref).max() <= 1e-11 * scale
    ar = cshift.real_part_arpack(K, C, M, sigma, nev)
    assert np.abs(ar - ref).max() <= 1e-10 * scale
    # planted: the nev nearest sigma are not the set (conjugate partners missing)
    near = oeig.nearest(dense, sigma, nev)
    assert np.abs(np.sort_complex(near) - np.sort_complex(ref)).max() > 1e-3 * scale


@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 8, 0)])
def test_maxwell_form_matches_dense_qz(p, ne, s):
    """Curl-conforming space, perfect conductor, C = alpha M + beta K: dense
    QZ on the element-assembled matrices, selection written out, against the
    Maxwell closed form with the null space; ARPACK agrees."""
    alpha, beta, nev = 0.2, 0.01, 10
    sigma = 0.0 + 6.0j
    K, M, C = hcurl.assemble_hcurl(p, ne, s, True, alpha, beta)
    dense = oeig.dense_qep(K, C, M)[0]
    ref = cshift.select(dense, sigma, nev)
    lam = cshift.maxwell_cshift(p, ne, s, alpha, beta, sigma, nev)
    scale = np.abs(ref).max()
    assert np.abs(lam - ref).max() <= 1e-10 * scale
    ar = cshift.real_part_arpack(K, C, M, sigma, nev)
    assert np.abs(ar - ref).max() <= 1e-9 * scale


def test_null_space_enters_near_the_origin():
    """A target near the origin on the curl-conforming space: the gradients'
    roots 0 and -alpha (multiplicity n_B^2 each) fill the selection; dropping
    the null space (planted) changes the set."""
    p, ne, s, alpha, beta, nev = 2, 8, 4, 0.2, 0.01, 6
    sigma = -0.15 + 0.3j
    K, M, C = hcurl.assemble_hcurl(p, ne, s, True, alpha, beta)
    ref = cshift.select(oeig.dense_qep(K, C, M)[0], sigma, nev)
    lam = cshift.maxwell_cshift(p, ne, s, alpha, beta, sigma, nev)
    assert np.abs(lam - ref).max() <= 1e-10
    assert np.all(np.minimum(np.abs(ref), np.abs(ref + alpha)) < 1e-8)
    nz = hcurl.maxwell_closed(p, ne, s, True, 1e-300, np.inf)
    r1, r2 = oeig.quad_roots(1.0, alpha + beta * nz, nz)
    planted = cshift.select(np.concatenate([r1, r2]), sigma, nev)
    assert np.abs(planted - ref).max() > 1e-3
