"""The divergence-conforming space and the vibroacoustic QEP (Sec. 2.2)
through the C ABI against the oracle: fig. MatPatterns sizes, K, M, C with
rigid and absorbing walls entrywise, the Cholesky solve of Q(sigma), the
undamped rigid cavity by spectrum slicing against the rotated Maxwell closed
form, and the damped QEP at a complex target against dense QZ and ARPACK's
real-part mode.  Every case prints its parameters first."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble as oasm
from oracle import cshift
from oracle import eigen as oeig
from oracle import hcurl, hdiv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig_matpatterns.json")
HDIV = 3
ALL = hdiv.LEFT | hdiv.RIGHT | hdiv.BOTTOM | hdiv.TOP


def _riga():
    from paper_2112_14064_amd import riga
    return riga


def _problem(p, ne, s, walls, alpha=0.0, beta=0.0, leaf=0):
    riga = _riga()
    print(f"[case] hdiv p={p} ne={ne} s={s} walls={walls} alpha={alpha} beta={beta} leaf={leaf}", flush=True)
    pr = riga.Problem(p, ne, s, leaf=leaf, space=HDIV, walls=walls)
    pr.assemble(alpha, beta)
    return pr


def _compare(pr, K, M, C):
    for which, A in ((0, K), (1, M), (2, C)):
        rowptr, col, val = pr.export_csr(which)
        assert np.array_equal(rowptr, A.indptr.astype(np.int64))
        assert np.array_equal(col, A.indices.astype(np.int32))
        scale = max(np.abs(A.data).max(), 1e-300)
        assert np.abs(val.cpu().numpy() - A.data).max() <= 1e-13 * scale, which


def test_fig_matpatterns_sizes():
    g = json.load(open(GOLD))
    for s, key in ((0, "iga"), (g["macro"], "riga")):
        pr = _problem(g["p"], g["ne"], s, ALL)
        assert (pr.ndof, pr.nnz) == (g[key]["N"], g[key]["nnz"])
        pr.close()


@pytest.mark.parametrize("p,ne,s,walls", [(2, 8, 4, 0), (3, 16, 8, hdiv.TOP), (3, 12, 0, hdiv.LEFT | hdiv.BOTTOM),
                                          (4, 16, 8, ALL), (2, 10, 5, hdiv.RIGHT | hdiv.TOP)])
def test_assembly_matches_oracle(p, ne, s, walls):
    pr = _problem(p, ne, s, walls, 0.7, 0.3)
    K, M, C = hdiv.assemble_hdiv(p, ne, s, walls, 0.7, 0.3)
    _compare(pr, K, M, C)
    pr.close()


@pytest.mark.parametrize("p,ne,s,walls,sigma", [(2, 16, 4, hdiv.TOP, 1.0), (3, 24, 8, ALL, 2.0),
                                                (3, 20, 0, hdiv.LEFT, 3.0)])
def test_solve_matches_sparse_solve(p, ne, s, walls, sigma):
    pr = _problem(p, ne, s, walls, 0.5, 0.2, leaf=8 if s == 0 else 0)
    pr.factor(sigma)
    K, M, C = hdiv.assemble_hdiv(p, ne, s, walls, 0.5, 0.2)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    rhs = np.random.default_rng(3).standard_normal((2, pr.ndof))
    x = pr.solve_q(torch.from_numpy(rhs)).cpu().numpy()
    xo = spla.spsolve(Q, rhs.T).reshape(pr.ndof, 2).T
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"  solve rel err {err:.2e}", flush=True)
    assert err < 1e-10
    pr.close()


@pytest.mark.parametrize("p,ne,s", [(2, 12, 4), (3, 16, 8), (3, 16, 0)])
def test_rigid_cavity_slices_match_rotated_maxwell(p, ne, s):
    """Rigid walls, no damping: K u = mu M u has the Maxwell values of the
    perfect-conductor curl-conforming space (the rotation)."""
    a, b = 5.0, 300.0
    pr = _problem(p, ne, s, 0)
    want = hcurl.maxwell_closed(p, ne, s, True, a, b)
    mu, U, eta, count, st, stats = pr.gep_slice(a, b, max_slice=24)
    print(f"  count {count} found {len(mu)} oracle {len(want)} status {st} stats {stats}", flush=True)
    assert st == 0 and count == len(want) == len(mu)
    assert (np.abs(mu - want) / want).max() <= 1e-10
    pr.close()


def _check_pairs(lam, X, eta, K, C, M, ref, tol=1e-10):
    assert len(lam) == len(ref)
    rel = np.abs(lam - ref) / np.abs(ref)
    print(f"  max rel err {rel.max():.2e}, max eta {eta.max():.2e}", flush=True)
    assert rel.max() <= tol
    assert eta.max() <= 1e-10
    U = X.cpu().numpy().T
    norms = (oeig.onenorm(K), oeig.onenorm(C), oeig.onenorm(M))
    for k in range(len(lam)):
        assert oeig.residual(K, C, M, lam[k], U[:, k], norms) <= 1e-10


def _nev_at_gap(ref_all, sigma, want):
    g = np.abs(cshift.psi(ref_all, sigma))
    n = want
    while n > 1 and g[n - 1] - g[n] <= 1e-6 * g[n - 1]:
        n -= 1
    return n


@pytest.mark.parametrize("p,ne,s,walls,sigma", [(2, 8, 4, hdiv.TOP, 0.5 + 6.0j), (3, 8, 0, hdiv.LEFT | hdiv.TOP, 0.3 + 8.0j)])
def test_damped_cavity_matches_dense_qz(p, ne, s, walls, sigma):
    alpha, beta = 0.5, 0.8
    pr = _problem(p, ne, s, walls, alpha, beta)
    K, M, C = hdiv.assemble_hdiv(p, ne, s, walls, alpha, beta)
    allref = cshift.select(oeig.dense_qep(K, C, M)[0], sigma, 40)
    nev = _nev_at_gap(allref, sigma, 12)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 36, block=2, seed=1)
    assert st == 0 and nconv == nev
    _check_pairs(lam, X, eta, K, C, M, allref[:nev], tol=1e-9)
    pr.close()


@pytest.mark.parametrize("s", [8, 0])
def test_damped_cavity_matches_arpack(s):
    """p=3 on 32x32 with an absorbing top wall: the pairs of largest |psi| at
    sigma = 0.5 + 7i against ARPACK's real-part mode on the oracle's matrices."""
    p, ne, walls, alpha, beta, sigma = 3, 32, hdiv.TOP, 0.5, 0.8, 0.5 + 7.0j
    pr = _problem(p, ne, s, walls, alpha, beta, leaf=8 if s == 0 else 0)
    K, M, C = hdiv.assemble_hdiv(p, ne, s, walls, alpha, beta)
    allref = cshift.real_part_arpack(K, C, M, sigma, 30)
    nev = _nev_at_gap(allref, sigma, 20)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 56, block=2, seed=2)
    assert st == 0 and nconv == nev
    _check_pairs(lam, X, eta, K, C, M, allref[:nev], tol=1e-9)
    pr.close()


def test_full_size_properties():
    """p=3 on 256x256, rIGA s=16, absorbing top wall: 40 pairs at sigma =
    0.5 + 7i converge with eta <= 1e-10, none grows (Re lam <= 0) and the
    returned set is closed under conjugation."""
    p, ne, s, walls, alpha, beta, sigma = 3, 256, 16, hdiv.TOP, 0.5, 0.8, 0.5 + 7.0j
    pr = _problem(p, ne, s, walls, alpha, beta)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(40, 80, block=2, seed=0)
    print(f"[full] hdiv: ndof {pr.ndof} nconv {nconv} status {st} max eta {eta.max():.2e} "
          f"max Re {lam.real.max():.2e} stats {pr.stats()}", flush=True)
    assert st == 0 and nconv == 40
    assert eta.max() <= 1e-10
    assert lam.real.max() <= 1e-10 * np.abs(lam).max()
    for x in lam[:38]:
        assert np.min(np.abs(lam - np.conj(x))) <= 1e-9 * np.abs(x)
    pr.close()
