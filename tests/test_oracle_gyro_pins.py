"""Pins of the gyroscopic oracle (oracle/gyro.py) against facts it does not
compute itself: the partition of unity and linear reproduction of B-splines
(for the 1-D skew matrix s_ij = int B_i B_j'), integration by parts, the
Kronecker factorisation of the 2-D form, the Hamiltonian spectrum of an
undamped gyroscopic pencil, LAPACK's dense QZ on small meshes and the
Rayleigh closed form at gx = 0; planted mistakes in the oracle's own
quantities must fail them."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble as oasm
from oracle import bspline as obs
from oracle import eigen as oeig
from oracle import gyro

CASES_1D = [(1, 6, 0), (2, 8, 4), (3, 12, 0), (3, 12, 4), (4, 10, 5)]


@pytest.mark.parametrize("p,ne,s", CASES_1D)
def test_skew_1d_partition_of_unity(p, ne, s):
    """sum_j B_j = 1, so sum_j int B_i B_j' = int B_i (sum_j B_j)' = 0."""
    S = gyro.assemble_1d_skew(p, ne, s, dirichlet=False)
    assert np.abs(S.sum(axis=1)).max() < 1e-14


@pytest.mark.parametrize("p,ne,s", CASES_1D)
def test_skew_1d_reproduces_linear_functions(p, ne, s):
    """sum_j g_j B_j(x) = x with the Greville abscissae g, so
    (S g)_i = int B_i dx = (t_{i+p+1} - t_i) / (p + 1); the transpose gives
    int B_i' x dx instead (the orientation of S is pinned)."""
    S = gyro.assemble_1d_skew(p, ne, s, dirichlet=False)
    g = gyro.greville(p, ne, s)
    kv = obs.knot_vector(p, ne, s)
    n = len(g)
    want = np.array([(kv[i + p + 1] - kv[i]) / (p + 1) for i in range(n)])
    assert np.abs(S @ g - want).max() < 1e-14
    # planted: the transposed matrix does not reproduce it
    assert np.abs(S.T @ g - want).max() > 1e-3


@pytest.mark.parametrize("p,ne,s", CASES_1D)
def test_skew_1d_integration_by_parts(p, ne, s):
    """int (B_i B_j' + B_i' B_j) = [B_i B_j]_0^1: only the first and last
    functions of an open knot vector are nonzero at the ends."""
    S = gyro.assemble_1d_skew(p, ne, s, dirichlet=False)
    n = S.shape[0]
    E = np.zeros((n, n))
    E[0, 0], E[-1, -1] = -1.0, 1.0
    assert np.abs(S + S.T - E).max() < 1e-14
    Sd = gyro.assemble_1d_skew(p, ne, s)
    assert np.abs(Sd + Sd.T).max() < 1e-14


@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 6, 0), (1, 5, 0)])
def test_2d_form_factorises(p, ne, s):
    """The element-by-element 2-D form equals gx M1 (x) S1 + gy S1 (x) M1 (x
    fastest), is skew-symmetric, and C carries alpha M + beta K on top."""
    gx, gy = 0.7, -0.4
    K, M, C = gyro.assemble_gyro(p, ne, s, 0.0, 0.0, gx, gy)
    K1, M1 = oasm.assemble_1d(p, ne, s)
    S1 = gyro.assemble_1d_skew(p, ne, s)
    G = gx * np.kron(M1, S1) + gy * np.kron(S1, M1)
    assert np.abs(C.toarray() - G).max() < 1e-15 * max(1.0, np.abs(G).max()) * 10
    assert abs(C + C.T).max() < 1e-15
    # planted: the derivative on the row function gives minus the form
    Gt = gx * np.kron(M1, S1.T) + gy * np.kron(S1.T, M1)
    assert np.abs(C.toarray() - Gt).max() > 0.1 * np.abs(G).max()
    K2, M2, C2 = gyro.assemble_gyro(p, ne, s, 0.05, 0.005, gx, gy)
    assert abs(C2 - (0.05 * M + 0.005 * K + C)).max() < 1e-15
    # the stored pattern is that of K (the library's tensor pattern)
    assert np.array_equal(C2.indptr, K.indptr) and np.array_equal(C2.indices, K.indices)


@pytest.mark.parametrize("p,ne,s,alpha,beta,gx", [(2, 8, 4, 0.05, 0.005, 0.8), (3, 6, 0, 0.0, 0.0, 1.5),
                                                   (2, 12, 4, 0.1, 0.01, 2.5), (1, 10, 0, 0.0, 0.0, 0.6)])
def test_closed_form_matches_dense_qz(p, ne, s, alpha, beta, gx):
    """The 1-D y-mode reduction against LAPACK's QZ on the full companion
    pencil of the element-assembled matrices (gy = 0)."""
    sigma, nev = 2.0, 12
    lam = gyro.gyro_closed(p, ne, s, alpha, beta, gx, sigma, nev)
    K, M, C = gyro.assemble_gyro(p, ne, s, alpha, beta, gx, 0.0)
    ref = oeig.nearest(oeig.dense_qep(K, C, M)[0], sigma, nev)
    assert np.abs(lam - ref).max() <= 1e-12 * np.abs(ref).max()
    # planted: dropping the gyroscopic term changes the eigenvalues
    lam0 = gyro.gyro_closed(p, ne, s, alpha, beta, 0.0, sigma, nev)
    assert np.abs(lam0 - ref).max() > 1e-3 * np.abs(ref).max()


def test_zero_gyration_is_the_rayleigh_closed_form():
    lam = gyro.gyro_closed(3, 24, 8, 0.05, 0.005, 0.0, 2.0, 16)
    ref, _ = oeig.rayleigh_closed(3, 24, 8, 0.05, 0.005, 2.0, 16)
    assert np.abs(lam - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("gy", [0.0, 1.3])
def test_undamped_gyroscopic_spectrum_is_hamiltonian(gy):
    """K, M SPD and C skew: every eigenvalue is purely imaginary and the
    spectrum is symmetric with respect to both axes."""
    K, M, C = gyro.assemble_gyro(2, 8, 4, 0.0, 0.0, 0.9, gy)
    lam = oeig.dense_qep(K, C, M)[0]
    scale = np.abs(lam).max()
    assert np.abs(lam.real).max() <= 1e-10 * scale
    for x in lam[:20]:
        assert np.min(np.abs(lam + x)) <= 1e-9 * scale
        assert np.min(np.abs(lam - np.conj(x))) <= 1e-9 * scale


def test_closed_form_search_covers_every_mode():
    """The mode cutoff of the closed form: with a strong gyration the nearest
    eigenvalues come from many y-modes; the result still equals dense QZ."""
    p, ne, s, gx = 2, 10, 0, 6.0
    lam = gyro.gyro_closed(p, ne, s, 0.0, 0.0, gx, 1.0, 20)
    K, M, C = gyro.assemble_gyro(p, ne, s, 0.0, 0.0, gx, 0.0)
    ref = oeig.nearest(oeig.dense_qep(K, C, M)[0], 1.0, 20)
    assert np.abs(lam - ref).max() <= 1e-12 * np.abs(ref).max()


def test_residual_of_dense_pairs():
    """Dense QZ pairs of the gyroscopic pencil have rounding-level scaled
    residuals under the oracle's residual (1-norms of the nonsymmetric C)."""
    K, M, C = gyro.assemble_gyro(2, 6, 3, 0.05, 0.005, 0.8, 0.3)
    lam, U = oeig.dense_qep(K, C, M)
    o = oeig.canonical_order(lam, 2.0)[:6]
    for k in o:
        assert oeig.residual(K, C, M, lam[k], U[:, k]) < 1e-12
    assert abs(oeig.onenorm(C) - np.abs(C.toarray()).sum(axis=0).max()) == 0.0
    assert sp.issparse(C)
