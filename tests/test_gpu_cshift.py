"""A complex target shift (riga_factor_complex, riga_solve_q_complex, riga_eigs
on the real part of the operator) through the C ABI against the oracle: the
complex solve against SciPy, eigenvalues against the closed forms (scalar
space and curl-conforming space with its null space), ARPACK's real-part mode
on small meshes, eigenvectors with the oracle's residual, the headline meshes
at full size, and the rejected combinations.  Every case prints its
parameters first."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble as oasm
from oracle import cshift
from oracle import eigen as oeig
from oracle import hcurl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H1, HCURL = 0, 1


def _riga():
    from paper_2112_14064_amd import riga
    return riga


def _problem(p, ne, s, space, alpha, beta, leaf=0):
    riga = _riga()
    print(f"[case] cshift p={p} ne={ne} s={s} space={space} alpha={alpha} beta={beta} leaf={leaf}", flush=True)
    pr = riga.Problem(p, ne, s, leaf=leaf, space=space)
    pr.assemble(alpha, beta)
    return pr


def _matrices(p, ne, s, space, alpha, beta):
    if space == H1:
        return oasm.assemble(p, ne, s, alpha, beta)
    return hcurl.assemble_hcurl(p, ne, s, True, alpha, beta)


def _nev_at_gap(ref_all, sigma, want):
    """The largest n <= want whose n-th and (n+1)-th |psi| differ (no cluster
    split at the cut)."""
    g = np.abs(cshift.psi(ref_all, sigma))
    n = want
    while n > 1 and g[n - 1] - g[n] <= 1e-6 * g[n - 1]:
        n -= 1
    return n


def _check(pr, lam, X, eta, K, C, M, ref, tol=1e-10):
    assert len(lam) == len(ref)
    rel = np.abs(lam - ref) / np.abs(ref)
    print(f"  max rel err {rel.max():.2e}, max eta {eta.max():.2e}", flush=True)
    assert rel.max() <= tol, (lam, ref)
    assert eta.max() <= 1e-10
    U = X.cpu().numpy().T
    norms = (oeig.onenorm(K), oeig.onenorm(C), oeig.onenorm(M))
    for k in range(len(lam)):
        assert oeig.residual(K, C, M, lam[k], U[:, k], norms) <= 1e-10
        assert abs(np.vdot(U[:, k], M @ U[:, k]) - 1.0) < 1e-10


@pytest.mark.parametrize("p,ne,s,space,sigma", [(2, 16, 4, H1, 0.5 + 7.0j), (3, 24, 0, H1, 0.0 + 5.0j),
                                                (2, 12, 4, HCURL, 0.0 + 6.0j), (3, 16, 8, HCURL, 1.0 + 4.0j)])
@pytest.mark.parametrize("nrhs", [1, 3, 6])
def test_complex_solve_matches_sparse_solve(p, ne, s, space, sigma, nrhs):
    alpha, beta = 0.05, 0.005
    pr = _problem(p, ne, s, space, alpha, beta, leaf=8 if s == 0 else 0)
    pr.factor(sigma)
    K, M, C = _matrices(p, ne, s, space, alpha, beta)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    rng = np.random.default_rng(nrhs)
    rhs = rng.standard_normal((nrhs, pr.ndof)) + 1j * rng.standard_normal((nrhs, pr.ndof))
    x = pr.solve_q_complex(torch.from_numpy(rhs)).cpu().numpy()
    xo = spla.spsolve(Q, rhs.T).reshape(pr.ndof, nrhs).T
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"  complex solve rel err {err:.2e}", flush=True)
    assert err < 1e-10
    pr.close()


@pytest.mark.parametrize("p,ne,s,sigma,block", [(3, 32, 8, 0.0 + 7.0j, 2), (2, 24, 0, 0.3 + 9.0j, 2),
                                                (3, 24, 8, 0.0 + 12.0j, 1), (4, 16, 4, 0.5 + 6.0j, 3)])
def test_scalar_eigs_match_closed_form(p, ne, s, sigma, block):
    alpha, beta = 0.05, 0.005
    pr = _problem(p, ne, s, H1, alpha, beta, leaf=8 if s == 0 else 0)
    allref = cshift.rayleigh_cshift(p, ne, s, alpha, beta, sigma, 64)
    nev = _nev_at_gap(allref, sigma, 16)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 48, block=block, seed=4)
    assert st == 0 and nconv == nev
    K, M, C = _matrices(p, ne, s, H1, alpha, beta)
    _check(pr, lam, X, eta, K, C, M, allref[:nev])
    pr.close()


def test_arpack_real_part_on_a_small_mesh():
    p, ne, s, sigma, alpha, beta = 2, 12, 4, 0.3 + 7.0j, 0.1, 0.01
    pr = _problem(p, ne, s, H1, alpha, beta)
    K, M, C = _matrices(p, ne, s, H1, alpha, beta)
    dense = oeig.dense_qep(K, C, M)[0]
    allref = cshift.select(dense, sigma, 40)
    nev = _nev_at_gap(allref, sigma, 12)
    ar = cshift.real_part_arpack(K, C, M, sigma, nev)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 36, block=2, seed=1)
    assert st == 0
    _check(pr, lam, X, eta, K, C, M, ar, tol=1e-9)
    pr.close()


@pytest.mark.parametrize("p,ne,s,sigma", [(2, 12, 4, 0.0 + 6.0j), (3, 16, 8, 0.0 + 9.0j), (3, 16, 0, 0.5 + 7.0j)])
def test_curl_conforming_eigs_match_closed_form(p, ne, s, sigma):
    """The conductive electromagnetic QEP on the curl-conforming space with
    the perfect conductor: a complex target reaches the physical modes past
    the gradients' 0 and -alpha."""
    alpha, beta = 0.2, 0.01
    pr = _problem(p, ne, s, HCURL, alpha, beta, leaf=8 if s == 0 else 0)
    allref = cshift.maxwell_cshift(p, ne, s, alpha, beta, sigma, 64)
    nev = _nev_at_gap(allref, sigma, 14)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 48, block=2, seed=2)
    assert st == 0 and nconv == nev
    K, M, C = _matrices(p, ne, s, HCURL, alpha, beta)
    _check(pr, lam, X, eta, K, C, M, allref[:nev])
    pr.close()


def test_rejections_and_return_to_a_real_shift():
    riga = _riga()
    pr = _problem(2, 12, 4, H1, 0.05, 0.005)
    pr.factor(0.0 + 5.0j)
    with pytest.raises(riga.RigaError):
        pr.solve_q(torch.ones((1, pr.ndof), dtype=torch.float64))
    with pytest.raises(riga.RigaError):
        pr.eigs(4, 20, flags=riga.RIGA_EIGS_TOAR)
    # a real factor ends the complex mode
    pr.factor(2.0)
    with pytest.raises(riga.RigaError):
        pr.solve_q_complex(torch.ones((1, pr.ndof), dtype=torch.complex128))
    lam, _, _, _, st = pr.eigs(8, 24, block=2)
    ref, _ = oeig.rayleigh_closed(2, 12, 4, 0.05, 0.005, 2.0, 8)
    assert st == 0 and np.abs(lam - ref).max() <= 1e-10 * np.abs(ref).max()
    # a gyroscopic damping has no complex target
    pr.assemble(0.05, 0.005, gyro=(0.5, 0.0))
    with pytest.raises(riga.RigaError):
        pr.factor(0.0 + 5.0j)
    pr.close()
    # a real shift on the curl-conforming space stays rejected
    ph = _problem(2, 8, 4, HCURL, 0.05, 0.005)
    ph.factor(2.0)
    with pytest.raises(riga.RigaError):
        ph.eigs(4, 20)
    ph.close()


@pytest.mark.parametrize("space,s", [(H1, 16), (H1, 0), (HCURL, 16)])
def test_full_size(space, s):
    """p=3 on 256x256 (the headline mesh; rIGA s=16 and IGA, and the
    curl-conforming space with the perfect conductor), Rayleigh 0.05 M +
    0.005 K, target sigma = 7i: the pairs of largest |psi| against the closed
    form, eta for all, sampled eigenvectors with the oracle's residual
    (matrices in Kronecker form on the scalar space)."""
    p, ne, alpha, beta, sigma = 3, 256, 0.05, 0.005, 0.0 + 7.0j
    pr = _problem(p, ne, s, space, alpha, beta)
    if space == H1:
        allref = cshift.rayleigh_cshift(p, ne, s, alpha, beta, sigma, 80)
    else:
        allref = cshift.maxwell_cshift(p, ne, s, alpha, beta, sigma, 80)
    nev = _nev_at_gap(allref, sigma, 40)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 80, block=2, seed=0)
    rel = np.abs(lam - allref[:nev]) / np.abs(allref[:nev])
    print(f"[full] cshift space={space} s={s}: ndof {pr.ndof} nev {nev} max rel {rel.max():.2e} "
          f"max eta {eta.max():.2e} stats {pr.stats()}", flush=True)
    assert st == 0 and nconv == nev
    assert rel.max() <= 1e-10
    assert eta.max() <= 1e-10
    pr.close()
