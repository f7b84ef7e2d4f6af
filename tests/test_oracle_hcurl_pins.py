"""Pins of the H(curl) oracle (oracle/hcurl.py) against facts it does not
compute itself: the printed sizes of fig. MatPatterns, the exactness of the
discrete de Rham sequence (K annihilates gradients, from the B-spline
derivative formula alone), the dimension of the gradient null space, dense
generalized eigenvalues on small meshes and the continuous Maxwell spectrum;
planted mistakes in the oracle's own quantities must fail them."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import hcurl
from oracle import space as ospace

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig_matpatterns.json")


def test_fig_matpatterns_from_assembled_matrices():
    """N and nnz of the assembled 64x64, p=4 H(curl) matrices (no boundary
    condition) equal the sizes printed under fig. MatPatterns, IGA and rIGA."""
    g = json.load(open(GOLD))
    for s, key in ((0, "iga"), (g["macro"], "riga")):
        K, M, C = hcurl.assemble_hcurl(g["p"], g["ne"], s, pec=False)
        assert K.shape[0] == g[key]["N"]
        assert K.nnz == g[key]["nnz"] == M.nnz
        assert (K.shape[0], K.nnz) == ospace.hcurl_counts(g["p"], g["ne"], s)


@pytest.mark.parametrize("p,ne,s,pec", [(2, 6, 3, True), (3, 8, 4, True), (3, 8, 0, False), (4, 8, 4, False),
                                        (2, 8, 0, True)])
def test_de_rham_exactness(p, ne, s, pec):
    """grad maps the scalar space into this one and K grad = 0 (rot grad = 0);
    the gradients fill the null space: rank G = its dimension."""
    K, M, C = hcurl.assemble_hcurl(p, ne, s, pec)
    G = hcurl.grad_matrix(p, ne, s, pec)
    assert abs(K @ G).max() <= 1e-13 * abs(K).max()
    assert np.linalg.matrix_rank(G.toarray()) == hcurl.null_dimension(p, ne, s, pec)
    # planted: the wrong sign of the coupling between the components breaks it
    nA = hcurl.spaces(p, ne, s, pec)[3]
    nB = hcurl.spaces(p, ne, s, pec)[4]
    base1 = nA * nB
    Kd = K.toarray()
    Kd[:base1, base1:] *= -1.0
    Kd[base1:, :base1] *= -1.0
    assert np.abs(Kd @ G.toarray()).max() > 1e-3 * np.abs(Kd).max()


@pytest.mark.parametrize("p,ne,s,pec", [(2, 6, 3, True), (3, 8, 4, True), (3, 8, 0, False), (4, 8, 4, True),
                                        (4, 8, 4, False)])
def test_closed_form_matches_dense_eigenvalues(p, ne, s, pec):
    K, M, C = hcurl.assemble_hcurl(p, ne, s, pec)
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max() and abs(M - M.T).max() <= 1e-15 * abs(M).max()
    w = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    scale = np.abs(w).max()
    zero = np.abs(w) < 1e-9 * scale
    assert zero.sum() == hcurl.null_dimension(p, ne, s, pec)
    nz = np.sort(w[~zero])
    cf = hcurl.maxwell_closed(p, ne, s, pec, 1e-9 * scale, np.inf)
    assert len(cf) == len(nz)
    assert np.abs(cf - nz).max() <= 1e-10 * scale
    # planted: C^0 (multiplicity p) knots in the degree-p factor change the rIGA spectrum
    if s:
        from oracle import bspline as obs
        kv = obs.knot_vector(p, ne, s)           # multiplicity p
        assert len(kv) != len(hcurl.spaces(p, ne, s, pec)[1])


def test_maxwell_spectrum_converges_to_the_continuous_one():
    """pi^2 (m^2 + n^2), m, n >= 0 not both zero: pi^2 twice, then 2 pi^2."""
    mu = hcurl.maxwell_closed(3, 32, 8, True, 1.0, 25.0)
    pi2 = np.pi ** 2
    assert np.allclose(mu[:3], [pi2, pi2, 2 * pi2], rtol=1e-7)


def test_mass_is_definite_and_stiffness_semidefinite():
    K, M, C = hcurl.assemble_hcurl(3, 6, 3, True, 0.05, 0.005)
    wm = np.linalg.eigvalsh(M.toarray())
    wk = np.linalg.eigvalsh(K.toarray())
    assert wm.min() > 0.0
    assert wk.min() > -1e-12 * wk.max()
    assert abs(C - (0.05 * M + 0.005 * K)).max() < 1e-15
    assert sp.issparse(C)
