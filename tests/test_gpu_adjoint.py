"""Adjoint d lam / d c_e of the HIP path against the oracle, the uniform-damping
closed form and central differences of GPU eigensolves."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import assemble as oasm
from oracle import eigen as oeig
from paper_2112_14064_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(p, ne, s, c, sigma, nev, alpha=0.0, m=24):
    from paper_2112_14064_amd import riga
    print(f"[case] adjoint p={p} ne={ne} s={s} sigma={sigma} nev={nev}", flush=True)
    pr = riga.Problem(p, ne, s)
    pr.assemble(alpha, 0.0, torch.from_numpy(np.ascontiguousarray(c)))
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, m, block=2, seed=4)
    assert st == 0 and nconv == nev
    return pr, lam, X


@pytest.mark.parametrize("p,ne,s", [(2, 12, 4), (3, 16, 8), (4, 12, 6)])
def test_adjoint_matches_oracle_elementwise(p, ne, s):
    sigma, nev = 2.0, 6
    c = W.lognormal_field(ne, 9)
    pr, lam, X = _solve(p, ne, s, c, sigma, nev)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(nev) + 1j * rng.standard_normal(nev)   # dL/dRe + i dL/dIm
    grad = pr.adjoint(lam, X, g).cpu().numpy()
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    U = X.cpu().numpy().T
    d = oadj.dlam_dc(p, ne, s, M, C, lam, U)            # (nev, ne, ne) complex
    ref = np.einsum("k,kij->ij", g.real, d.real) + np.einsum("k,kij->ij", g.imag, d.imag)
    assert np.abs(grad - ref).max() <= 1e-10 * np.abs(ref).max()
    pr.close()


def test_adjoint_uniform_closed_form():
    """C = c M: lam^2 + c lam + mu = 0, so d lam/dc = -lam/(2 lam + c); the
    element sensitivities sum to it since sum_e M_e = M."""
    p, ne, s, sigma, nev, cval = 3, 16, 8, 2.0, 8, 0.07
    pr, lam, X = _solve(p, ne, s, np.full((ne, ne), cval), sigma, nev)
    grad = pr.adjoint(lam, X, np.ones(nev, dtype=complex)).cpu().numpy()
    want = np.sum(np.real(-lam / (2 * lam + cval)))
    assert abs(grad.sum() - want) <= 1e-10 * abs(want)
    pr.close()


def test_adjoint_central_differences():
    p, ne, s, sigma, nev = 2, 12, 4, 2.0, 6
    c = W.lognormal_field(ne, 13)
    pr, lam, X = _solve(p, ne, s, c, sigma, nev)
    grad = pr.adjoint(lam, X, np.ones(nev, dtype=complex)).cpu().numpy()
    pr.close()

    def L(cc):
        pr2, l2, _ = _solve(p, ne, s, cc, sigma, nev)
        pr2.close()
        return np.sum(l2.real)

    h = 1e-4
    for e in [(0, 0), (5, 7), (11, 3)]:
        cp, cm = c.copy(), c.copy()
        cp[e] += h
        cm[e] -= h
        fd = (L(cp) - L(cm)) / (2 * h)
        assert abs(grad[e] - fd) <= 1e-5 * abs(fd) + 1e-9, (e, grad[e], fd)


def test_autograd_function_matches_adjoint():
    from paper_2112_14064_amd import riga
    from paper_2112_14064_amd.autograd import qep_eigenvalues
    p, ne, s, sigma, nev = 2, 12, 4, 2.0, 6
    c = torch.from_numpy(W.lognormal_field(ne, 17)).cuda().requires_grad_(True)
    pr = riga.Problem(p, ne, s)
    lam = qep_eigenvalues(c, pr, sigma, nev, m=24)
    loss = lam.real.sum()
    loss.backward()
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c.detach().cpu().numpy())
    lam_o = oeig.nearest(oeig.dense_qep(K, C, M)[0], sigma, nev)
    assert np.abs(lam.detach().cpu().numpy() - lam_o).max() < 1e-10 * np.abs(lam_o).max()
    pr2, lam2, X2 = _solve(p, ne, s, c.detach().cpu().numpy(), sigma, nev)
    g2 = pr2.adjoint(lam2, X2, np.ones(nev, dtype=complex)).cpu().numpy()
    # two independent solves (different start blocks): eigenvectors agree to ~1e-12
    assert np.abs(c.grad.cpu().numpy() - g2).max() <= 1e-9 * np.abs(g2).max()
    pr.close()
    pr2.close()


def test_adjoint_full_size():
    """p=3 on 512x512 (330,625 dofs, 262,144 elements), 20 eigenvalues near
    sigma=2, L = sum Re lam.  Sampled elements against the oracle's formula
    with the returned eigenvectors; central differences of full GPU solves on
    32 seeded elements (h = 1e-2 for the relative check; the FP64 resolution of
    L limits smaller steps), and the uniform-direction identity."""
    P = W.cfg_adjoint()
    pr, lam, X = _solve(P.p, P.ne, P.hyper_every, P.c_elem, P.sigma, P.nev, m=P.m)
    grad = pr.adjoint(lam, X, np.ones(P.nev, dtype=complex)).cpu().numpy()
    assert np.all(np.isfinite(grad))
    print("[full] solve + adjoint done; sampling the oracle formula", flush=True)
    # oracle formula on 48 sampled elements with the same eigenvectors
    from oracle.assemble import element_mass_2d
    U = X.cpu().numpy().T
    # denominators u^T (2 lam M + C) u through the library's assembled M, C
    rowptr, col, mv = pr.export_csr(1)
    _, _, cv = pr.export_csr(2)
    import scipy.sparse as sp
    N = pr.ndof
    M = sp.csr_matrix((mv.cpu().numpy(), col, rowptr), shape=(N, N))
    Cm = sp.csr_matrix((cv.cpu().numpy(), col, rowptr), shape=(N, N))
    den = np.array([U[:, k] @ (2 * lam[k] * (M @ U[:, k]) + Cm @ U[:, k]) for k in range(P.nev)])
    rng = np.random.default_rng(5)
    for e in rng.choice(P.ne * P.ne, 48, replace=False):
        ey, ex = divmod(int(e), P.ne)
        dofs, Me = element_mass_2d(P.p, P.ne, P.hyper_every, ex, ey)
        ok = dofs >= 0
        q = np.array([U[dofs[ok], k] @ Me[np.ix_(ok, ok)] @ U[dofs[ok], k] for k in range(P.nev)])
        ref = np.sum(np.real(-lam * q / den))
        assert abs(grad[ey, ex] - ref) <= 1e-9 * np.abs(grad).max()
    pr.close()
    print("[full] sampled elements agree; central differences", flush=True)
    # central differences of full solves
    def L(cc):
        pr2, l2, _ = _solve(P.p, P.ne, P.hyper_every, cc, P.sigma, P.nev, m=P.m)
        pr2.close()
        return np.sum(l2.real)
    els = W.fd_elements(P.ne, 32, seed=2)
    h = 1e-2
    fd = []
    for e in els:
        ey, ex = divmod(int(e), P.ne)
        cp, cm = P.c_elem.copy(), P.c_elem.copy()
        cp[ey, ex] += h
        cm[ey, ex] -= h
        fd.append((L(cp) - L(cm)) / (2 * h))
        print(f"[full] fd element {int(e)} done", flush=True)
    fd = np.array(fd)
    ga = np.array([grad[divmod(int(e), P.ne)] for e in els])
    print("adjoint vs FD: max abs diff", np.abs(ga - fd).max(), "max |fd|", np.abs(fd).max(), flush=True)
    assert np.abs(ga - fd).max() <= 1e-5 * np.abs(fd).max() + 4e-13 / h
