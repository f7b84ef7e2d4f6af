"""Pins of the oracle's C = 0 generalized eigenproblem and inertia counts
(Sec. 4.1.4, spectrum slicing) against mathematics: Sylvester's law on a
diagonal pencil worked by hand, dense LAPACK solves of the assembled pencil
(symmetric-definite eigensolver and the Bunch-Kaufman factorization, two
independent routes) against the Kronecker-sum closed form, and planted
mistakes that the pins catch.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble as oasm
from oracle import eigen as oeig
from oracle import gep as ogep


def test_inertia_of_a_diagonal_pencil_by_hand():
    """K = diag(1, 4, 9, 16), M = diag(1, 2, 1, 4): eigenvalues 1, 2, 9, 4, so
    K - s M has exactly #{mu < s} negative diagonal entries."""
    K = np.diag([1.0, 4.0, 9.0, 16.0])
    M = np.diag([1.0, 2.0, 1.0, 4.0])
    for s, want in ((0.5, 0), (1.5, 1), (3.0, 2), (5.0, 3), (9.5, 4)):
        assert ogep.inertia_dense(K, M, s) == want
    mu, U = ogep.gep_dense(K, M)
    assert np.allclose(mu, [1.0, 2.0, 4.0, 9.0], rtol=0, atol=1e-14)
    assert np.allclose(U.T @ M @ U, np.eye(4), atol=1e-14)


@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 8, 0), (2, 12, 4)])
def test_closed_form_matches_dense_generalized_solve(p, ne, s):
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    mu, _ = ogep.gep_dense(K, M)
    lo, hi = mu[3] * 0.999, mu[min(len(mu) - 1, 40)] * 1.0001
    got = ogep.gep_closed(p, ne, s, lo, hi)
    want = mu[(mu >= lo) & (mu < hi)]
    assert len(got) == len(want)
    assert np.allclose(got, want, rtol=1e-11, atol=0)


@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 10, 0)])
def test_inertia_counts_agree(p, ne, s):
    """nu(K - s M) from the indefinite factorization equals the closed-form
    count, at shifts between eigenvalues, just below and just above one, and
    below the whole spectrum."""
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    mu, _ = ogep.gep_dense(K, M)
    # midpoints of gaps between distinct eigenvalues (the square has double ones)
    gaps = [k for k in range(len(mu) - 1) if mu[k + 1] - mu[k] > 1e-6 * mu[k + 1]]
    shifts = [0.5 * mu[0], 0.5 * (mu[gaps[2]] + mu[gaps[2] + 1]), mu[9] * (1 - 1e-7), mu[9] * (1 + 1e-7),
              0.5 * (mu[gaps[8]] + mu[gaps[8] + 1])]
    for sh in shifts:
        a = ogep.inertia_dense(K, M, sh)
        b = ogep.count_below(p, ne, s, sh)
        assert a == b == int(np.sum(mu < sh)), (sh, a, b)


def test_multiplicity_two_is_counted_twice():
    """mu_12 = mu_21 on the square: the closed form returns both copies, and
    the inertia jump across the value is 2."""
    p, ne, s = 2, 8, 4
    mu1 = oeig.mu_1d(p, ne, s)
    m12 = mu1[0] + mu1[1]
    got = ogep.gep_closed(p, ne, s, m12 * (1 - 1e-9), m12 * (1 + 1e-9))
    assert len(got) == 2
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    assert ogep.inertia_dense(K, M, m12 * (1 + 1e-7)) - ogep.inertia_dense(K, M, m12 * (1 - 1e-7)) == 2


def test_gep_residual_hand_computed():
    """K = [[2, 1], [1, 3]] (1-norm 4), M = I (1-norm 1), mu = 1, u = [1, 0]:
    K u - u = [1, 1], so eta = sqrt(2) / ((4 + 1) * 1)."""
    K = np.array([[2.0, 1.0], [1.0, 3.0]])
    M = np.eye(2)
    assert ogep.gep_residual(K, M, 1.0, np.array([1.0, 0.0])) == pytest.approx(np.sqrt(2.0) / 5.0, rel=1e-15)


def test_pins_catch_slicing_mistakes(monkeypatch):
    """Counting only i <= j (no multiplicity), or <= instead of < at the upper
    end, changes the counts the pins compare."""
    p, ne, s = 2, 8, 4
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    mu, _ = ogep.gep_dense(K, M)
    gaps = [k for k in range(len(mu) - 1) if mu[k + 1] - mu[k] > 1e-6 * mu[k + 1]]
    sh = 0.5 * (mu[gaps[8]] + mu[gaps[8] + 1])
    mu1 = oeig.mu_1d(p, ne, s)
    half = sum(1 for i in range(len(mu1)) for j in range(i, len(mu1)) if mu1[i] + mu1[j] < sh)
    assert half != ogep.inertia_dense(K, M, sh)
    # an upper end placed exactly on an eigenvalue: [a, b) leaves it out
    m = ogep.gep_closed(p, ne, s, 0.0, np.inf)[9]
    assert m not in ogep.gep_closed(p, ne, s, 0.0, m)
    assert ogep.count_below(p, ne, s, m) == int(np.sum(ogep.gep_closed(p, ne, s, 0.0, np.inf) < m))
