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


def _secant_quotients(lp, Xp, lm, Xm, M, C0, dofs, Me, dc_minus):
    """(lam_k(c + h e) - lam_k(c - h e)) / (2h) for every k, from the two
    perturbed eigenpairs, without subtracting the eigenvalues.

    With Q_pm(lam) = lam^2 M + lam C_pm + K and C_+ - C_- = 2h M_e:
    x_-^T Q_+(lam_+) x_+ = 0 and x_-^T Q_-(lam_-) = 0 (complex-symmetric pencil)
    give, after Q_-(lam_+) - Q_-(lam_-) = (lam_+ - lam_-) [(lam_+ + lam_-) M + C_-],
        lam_+ - lam_- = -2h lam_+ x_-^T M_e x_+ / x_-^T [(lam_+ + lam_-) M + C_-] x_+,
    an exact identity for exact pairs.  C_- = C0 + dc_minus M_e."""
    MX = M @ Xp
    CX = C0 @ Xp
    out = np.zeros(len(lp), dtype=complex)
    ok = dofs >= 0
    d = dofs[ok]
    Mee = Me[np.ix_(ok, ok)]
    for k in range(len(lp)):
        xm, xp = Xm[:, k], Xp[:, k]
        num = xm[d] @ Mee @ xp[d]
        den = xm @ ((lp[k] + lm[k]) * MX[:, k] + CX[:, k]) + dc_minus * num
        out[k] = -lp[k] * num / den
    return out


@pytest.mark.timeout(900)
def test_adjoint_full_size_central_differences_h1e6():
    """The configured check of the p=3 512x512 workload: central differences
    with h = 1e-6 on 32 seeded elements of L = sum Re lam over the 20
    eigenvalues nearest sigma = 2, each L(c +- h e) from a full GPU solve.  The
    difference of the two solves' eigenvalues is taken through the two-pencil
    identity of _secant_quotients (oracle M, C and M_e), which is the central
    quotient itself without the cancellation that limits a plain subtraction
    to ~eps |lam| / h.  The identity is first checked against plain subtraction
    at h = 1e-2, where both are resolved."""
    from oracle.assemble import element_mass_2d
    P = W.cfg_adjoint()
    pr, lam, X = _solve(P.p, P.ne, P.hyper_every, P.c_elem, P.sigma, P.nev, m=P.m)
    grad = pr.adjoint(lam, X, np.ones(P.nev, dtype=complex)).cpu().numpy()
    pr.close()
    print("[full] oracle assembly of M and C", flush=True)
    K, M, C0 = oasm.assemble(P.p, P.ne, P.hyper_every, 0.0, 0.0, P.c_elem)
    del K

    def solve(cc):
        pr2, l2, X2 = _solve(P.p, P.ne, P.hyper_every, cc, P.sigma, P.nev, m=P.m)
        U2 = X2.cpu().numpy().T
        pr2.close()
        return l2, U2

    def quotients(e, h):
        ey, ex = divmod(int(e), P.ne)
        cp, cm = P.c_elem.copy(), P.c_elem.copy()
        cp[ey, ex] += h
        cm[ey, ex] -= h
        two_h = cp[ey, ex] - cm[ey, ex]          # exact spacing of the two FP64 inputs
        lp, Xp = solve(cp)
        lm, Xm = solve(cm)
        dofs, Me = element_mass_2d(P.p, P.ne, P.hyper_every, ex, ey)
        q = _secant_quotients(lp, Xp, lm, Xm, M, C0, dofs, Me, cm[ey, ex] - P.c_elem[ey, ex])
        plain = (np.sum(lp.real) - np.sum(lm.real)) / two_h
        return float(np.sum(q.real)), float(plain), float(abs(np.sum(lp.real))), float(np.sum(np.abs(lp))), two_h

    els = W.fd_elements(P.ne, 32, seed=2)
    # the identity against plain subtraction where both are resolved
    # plain subtraction carries the solves' eigenvalue errors (about 1e-14
    # relative each) divided by the step
    for e in els[:4]:
        qi, qp, _, sum_abs, two_h = quotients(e, 1e-2)
        print(f"[full] h=1e-2 element {int(e)}: identity {qi:.12e} plain {qp:.12e}", flush=True)
        assert abs(qi - qp) <= 1e-8 * abs(qp) + 2e-14 * sum_abs / two_h
    # the configured step
    h = 1e-6
    fd, plain, Ls = [], [], []
    for e in els:
        qi, qp, Lv, _, _ = quotients(e, h)
        fd.append(qi)
        plain.append(qp)
        Ls.append(Lv)
        print(f"[full] h=1e-6 element {int(e)}: fd {qi:.6e} (plain subtraction {qp:.6e})", flush=True)
    fd = np.array(fd)
    ga = np.array([grad[divmod(int(e), P.ne)] for e in els])
    eps = np.finfo(float).eps
    bound = 1e-5 * np.abs(fd).max() + 4 * eps * max(Ls) / h
    print(f"adjoint vs central differences (h=1e-6): max abs diff {np.abs(ga - fd).max():.3e}, "
          f"max |fd| {np.abs(fd).max():.3e}, bound {bound:.3e}; plain subtraction max diff "
          f"{np.abs(ga - np.array(plain)).max():.3e}", flush=True)
    assert np.abs(ga - fd).max() <= bound
