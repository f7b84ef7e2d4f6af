"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case prints its parameters before touching the GPU so that a failure
names its case.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble as oasm
from oracle import eigen as oeig
from paper_2112_14064_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _riga():
    from paper_2112_14064_amd import riga
    return riga


def _problem(p, ne, s, alpha=0.0, beta=0.0, c=None, leaf=0):
    riga = _riga()
    print(f"[case] p={p} ne={ne} s={s} alpha={alpha} beta={beta} elem={c is not None} leaf={leaf}", flush=True)
    pr = riga.Problem(p, ne, s, leaf=leaf)
    pr.assemble(alpha, beta, None if c is None else torch.from_numpy(np.ascontiguousarray(c)))
    return pr


ASM_CASES = [(2, 16, 4), (3, 24, 8), (4, 16, 8), (3, 20, 0), (1, 8, 0), (2, 12, 12), (5, 12, 6), (3, 40, 0)]


@pytest.mark.parametrize("p,ne,s", ASM_CASES)
def test_assembly_matches_oracle(p, ne, s):
    c = W.lognormal_field(ne, 11)
    pr = _problem(p, ne, s, 0.07, 0.003, c)
    K, M, C = oasm.assemble(p, ne, s, 0.07, 0.003, c)
    for which, A in ((0, K), (1, M), (2, C)):
        rowptr, col, val = pr.export_csr(which)
        assert np.array_equal(rowptr, A.indptr.astype(np.int64))
        assert np.array_equal(col, A.indices.astype(np.int32))
        v = val.cpu().numpy()
        scale = np.abs(A.data).max()
        assert np.abs(v - A.data).max() <= 1e-13 * scale, which
    pr.close()


SOLVE_CASES = [(2, 16, 4, 1.0), (3, 32, 8, 2.0), (4, 24, 8, 5.0), (3, 24, 0, 2.0), (2, 10, 10, 0.7),
               (3, 64, 16, 2.0), (2, 33, 0, 1.5)]


@pytest.mark.parametrize("p,ne,s,sigma", SOLVE_CASES)
@pytest.mark.parametrize("nrhs", [1, 2, 4])
def test_solve_q_matches_sparse_solve(p, ne, s, sigma, nrhs):
    c = W.lognormal_field(ne, 3)
    pr = _problem(p, ne, s, 0.05, 0.005, c, leaf=8 if s == 0 else 0)
    pr.factor(sigma)
    K, M, C = oasm.assemble(p, ne, s, 0.05, 0.005, c)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    b = W.random_rhs(pr.ndof, nrhs, seed=nrhs)
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    xo = spla.spsolve(Q, b.T).reshape(pr.ndof, nrhs).T
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert err < 1e-11, err
    # residual of the GPU solution with the oracle matrix
    r = (Q @ x.T - b.T)
    assert np.abs(r).max() / np.abs(b).max() < 1e-11
    pr.close()


@pytest.mark.parametrize("p,ne,s,sigma", [(2, 16, 4, 1.0), (3, 24, 0, 2.0)])
def test_apply_op_matches_block_operator(p, ne, s, sigma):
    pr = _problem(p, ne, s, 0.1, 0.01)
    pr.factor(sigma)
    K, M, C = oasm.assemble(p, ne, s, 0.1, 0.01)
    n = pr.ndof
    v = W.start_block(n, 3, seed=4)
    r = pr.apply_op(torch.from_numpy(v)).cpu().numpy()
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    for q in range(3):
        vu, vl = v[q, :n], v[q, n:]
        ru = -spla.spsolve(Q, sigma * (M @ vu) + C @ vu + M @ vl)
        rl = sigma * ru + vu
        ref = np.concatenate([ru, rl])
        assert np.abs(r[q] - ref).max() / np.abs(ref).max() < 1e-11
    pr.close()


def _check_pairs(pr, lam, X, eta, K, C, M, ref, nev, sigma, tol=1e-10):
    assert len(lam) == nev
    rel = np.abs(lam - ref) / np.abs(ref)
    assert rel.max() <= tol, (rel.max(), lam, ref)
    assert np.all(eta <= 1e-10), eta
    if X is not None:
        U = X.cpu().numpy().T
        norms = (oeig.onenorm(K), oeig.onenorm(C), oeig.onenorm(M))
        for k in range(nev):
            u = U[:, k]
            assert oeig.residual(K, C, M, lam[k], u, norms) <= 1e-10
            assert abs(np.vdot(u, M @ u) - 1.0) < 1e-10
            # an entry of largest modulus (ties within rounding: symmetric modes
            # have several) is real positive
            big = np.flatnonzero(np.abs(u) >= (1 - 1e-9) * np.abs(u).max())
            assert any(abs(u[i].imag) <= 1e-12 * abs(u[i]) and u[i].real > 0 for i in big)


def test_eigs_small_config_rayleigh():
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0)
    assert st == 0 and nconv == P.nev
    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    K, M, C = oasm.assemble(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    lam_d = oeig.nearest(oeig.dense_qep(K, C, M)[0], P.sigma, P.nev)
    assert np.abs(ref - lam_d).max() / np.abs(ref).max() < 1e-12
    _check_pairs(pr, lam, X, eta, K, C, M, ref, P.nev, P.sigma)
    pr.close()


@pytest.mark.parametrize("block", [1, 2, 3, 4])
def test_eigs_element_damping_dense(block):
    p, ne, s, sigma, nev = 3, 12, 4, 2.0, 8
    c = W.lognormal_field(ne, 5)
    pr = _problem(p, ne, s, 0.0, 0.0, c)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 24, block=block, seed=1)
    assert st == 0
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    ref = oeig.nearest(oeig.dense_qep(K, C, M)[0], sigma, nev)
    _check_pairs(pr, lam, X, eta, K, C, M, ref, nev, sigma)
    pr.close()


@pytest.mark.parametrize("p,ne,s,leaf", [(3, 32, 0, 8), (2, 24, 0, 16), (3, 32, 8, 0), (4, 16, 4, 0)])
def test_eigs_iga_and_riga_closed_form(p, ne, s, leaf):
    sigma, nev, a, b = 2.0, 12, 0.05, 0.005
    pr = _problem(p, ne, s, a, b, leaf=leaf)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 32, block=2, seed=3)
    assert st == 0
    ref, _ = oeig.rayleigh_closed(p, ne, s, a, b, sigma, nev)
    K, M, C = oasm.assemble(p, ne, s, a, b)
    _check_pairs(pr, lam, X, eta, K, C, M, ref, nev, sigma)
    pr.close()


def test_eigs_start_block_spanning_invariant_subspace():
    """A start block that spans an exact invariant subspace makes the first
    block step break down; the solver must still return the nearest pairs."""
    P = W.cfg_small()
    K, M, C = oasm.assemble(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    lam_all, U = oeig.dense_qep(K, C, M)
    o = oeig.canonical_order(lam_all, P.sigma)
    lam0, u0 = lam_all[o[0]], U[:, o[0]]
    x = np.concatenate([u0, lam0 * u0])
    v0 = np.stack([x.real, x.imag])
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, v0=torch.from_numpy(v0))
    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    _check_pairs(pr, lam, X, eta, K, C, M, ref, P.nev, P.sigma)
    pr.close()


def test_eigs_maxit_warning():
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.nev + 2, block=2, maxit=1, tol=1e-14)
    assert st == 1  # RIGA_WARN_NOT_CONVERGED
    assert 0 <= nconv <= P.nev
    pr.close()


def test_eigs_bitwise_deterministic():
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    a = pr.eigs(P.nev, P.m, block=2, seed=7)
    b = pr.eigs(P.nev, P.m, block=2, seed=7)
    assert np.array_equal(a[0], b[0])
    assert torch.equal(a[1], b[1])
    pr.close()


def test_not_spd_reports_pivot():
    riga = _riga()
    pr = _problem(2, 8, 4, -100.0, 0.0)
    with pytest.raises(riga.RigaError) as e:
        pr.factor(5.0)
    assert e.value.status == riga.RIGA_ERR_NOT_SPD
    assert 0 <= e.value.bad_pivot < pr.ndof
    with pytest.raises(riga.RigaError):
        pr.solve_q(torch.zeros((1, pr.ndof), dtype=torch.float64))
    pr.close()


def test_graph_replays_match_eager_launches():
    """Block steps replayed from captured HIP graphs give bitwise the results of
    eager launches, across several solves on one handle (each replay follows
    the previous solve's host work and synchronisations)."""
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    eager = pr.eigs(P.nev, P.m, block=2, seed=11, flags=1)
    for _ in range(3):
        rep = pr.eigs(P.nev, P.m, block=2, seed=11)
        assert np.array_equal(rep[0], eager[0])
        assert torch.equal(rep[1], eager[1])
    pr.close()


def test_host_checked_path_matches_closed_form():
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0, flags=2)
    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    K, M, C = oasm.assemble(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    _check_pairs(pr, lam, X, eta, K, C, M, ref, P.nev, P.sigma)
    pr.close()


@pytest.mark.parametrize("s", [16, 0])
def test_headline_workload_full_size(s):
    """p=3 on 256x256, rIGA with C^0 hyperplanes every 16 elements (82,369 dofs)
    and IGA (66,049 dofs), Rayleigh 0.05 M + 0.005 K, the 40 eigenpairs nearest
    sigma = 2 with subspace 80: every eigenvalue against the closed form
    (Kronecker sum of the 1-D pencil), the library's eta for all pairs and the
    oracle's eta, M-normalisation and phase for sampled eigenvectors."""
    P = W.cfg_riga_vs_iga(s)
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    assert pr.ndof == (82369 if s else 66049)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0)
    assert st == 0 and nconv == P.nev
    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    rel = np.abs(lam - ref) / np.abs(ref)
    print(f"[full] {P.name}: max rel err {rel.max():.2e}, max eta {eta.max():.2e}", flush=True)
    assert rel.max() <= 1e-10
    assert eta.max() <= 1e-10
    K, M, C = oasm.assemble(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    norms = (oeig.onenorm(K), oeig.onenorm(C), oeig.onenorm(M))
    U = X.cpu().numpy().T
    for k in np.random.default_rng(2).choice(P.nev, 6, replace=False):
        u = U[:, k]
        assert oeig.residual(K, C, M, lam[k], u, norms) <= 1e-10
        assert abs(np.vdot(u, M @ u) - 1.0) < 1e-10
    pr.close()


def test_reassembly_and_subspace_change_on_one_handle():
    """Captured block steps must not outlive the operator they were recorded
    for: on one handle, a smaller subspace after a larger one, new Rayleigh
    coefficients at the same shift, and a switch between Rayleigh and element
    damping at the same shift each give the closed form / dense QZ."""
    p, ne, s, sigma, nev = 2, 16, 4, 1.0, 6
    pr = _problem(p, ne, s, 0.1, 0.01)
    pr.factor(sigma)
    for m in (40, 20):
        lam, X, eta, nconv, st = pr.eigs(nev, m, block=2, seed=3)
        ref, _ = oeig.rayleigh_closed(p, ne, s, 0.1, 0.01, sigma, nev)
        print(f"[case] m={m} max rel err {np.max(np.abs(lam - ref) / np.abs(ref)):.2e}", flush=True)
        assert st == 0 and np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    for a, b in ((0.3, 0.002), (0.02, 0.03)):
        pr.assemble(a, b)
        pr.factor(sigma)
        lam, X, eta, nconv, st = pr.eigs(nev, 20, block=2, seed=3)
        ref, _ = oeig.rayleigh_closed(p, ne, s, a, b, sigma, nev)
        print(f"[case] alpha={a} beta={b} max rel err {np.max(np.abs(lam - ref) / np.abs(ref)):.2e}", flush=True)
        assert st == 0 and np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    c = W.lognormal_field(ne, 21)
    pr.assemble(0.0, 0.0, torch.from_numpy(c))
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 20, block=2, seed=3)
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    ref = oeig.nearest(oeig.dense_qep(K, C, M)[0], sigma, nev)
    assert st == 0 and np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    pr.assemble(0.1, 0.01)
    pr.factor(sigma)
    lam, X, eta, nconv, st = pr.eigs(nev, 20, block=2, seed=3)
    ref, _ = oeig.rayleigh_closed(p, ne, s, 0.1, 0.01, sigma, nev)
    assert st == 0 and np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    pr.close()


def test_stats_follow_the_cost_model():
    """Per-phase counters of riga_stats (eq. Cost): the factorization flops are
    the symbolic count, the eliminations 4 nnz(L) per vector, the products
    2 nnz per product, and every phase that ran has work."""
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0)
    s_ = pr.stats()
    inf = pr.info
    _, cc, nz, fl = _riga().riga_symbolic(P.p, P.ne, P.hyper_every)
    assert inf["factor_nnz"] == nz and inf["factor_flops"] == fl
    assert s_["flops"]["factor"] == fl
    assert s_["flops"]["fb"] == pytest.approx(s_["n_fb"] * 4.0 * nz)
    assert s_["flops"]["mv"] == pytest.approx(s_["n_mv"] * 2.0 * inf["nnz"])
    assert s_["flops"]["vv"] == pytest.approx(s_["n_vv"] * 2.0 * pr.ndof)
    for ph in ("assemble", "factor", "fb", "mv", "vv", "restart", "post"):
        assert s_["bytes"][ph] > 0, ph
    assert s_["bytes"]["ir"] == 0 and s_["flops"]["ir"] == 0
    pr.close()
