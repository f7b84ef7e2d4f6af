"""Mixed-precision factor through the C ABI: FP32 fronts (FP32 MFMA products
and accumulation) below the top tree levels, FP64 top levels, and FP64
iterative refinement of every solve; checked against the CPU oracle and
against the FP64 path.

Every case prints its parameters before touching the GPU so that a failure
names its case.
"""
import numpy as np
import pytest
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
    print(f"[case] mixed p={p} ne={ne} s={s} alpha={alpha} beta={beta} elem={c is not None} leaf={leaf}",
          flush=True)
    pr = riga.Problem(p, ne, s, leaf=leaf)
    pr.assemble(alpha, beta, None if c is None else torch.from_numpy(np.ascontiguousarray(c)))
    return pr


MIXED_SOLVE = [(2, 16, 4, 1.0), (3, 32, 8, 2.0), (4, 24, 8, 5.0), (3, 24, 0, 2.0), (3, 64, 16, 2.0),
               (4, 64, 32, 5.0)]


@pytest.mark.parametrize("p,ne,s,sigma", MIXED_SOLVE)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_mixed_solve_matches_sparse_solve(p, ne, s, sigma, nrhs):
    c = W.lognormal_field(ne, 3)
    pr = _problem(p, ne, s, 0.05, 0.005, c, leaf=8 if s == 0 else 0)
    pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=4)
    assert pr.ir_sweeps() == 4
    K, M, C = oasm.assemble(p, ne, s, 0.05, 0.005, c)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    b = W.random_rhs(pr.ndof, nrhs, seed=nrhs)
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    xo = spla.spsolve(Q, b.T).reshape(pr.ndof, nrhs).T
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert err < 1e-11, err
    r = Q @ x.T - b.T
    assert np.abs(r).max() / np.abs(b).max() < 1e-11
    pr.close()


@pytest.mark.parametrize("p,ne,s,sigma", [(3, 32, 8, 2.0), (4, 64, 32, 5.0)])
def test_unrefined_solve_carries_fp32_error(p, ne, s, sigma):
    """With no refinement the FP32 fronts show: the error is far above FP64
    rounding yet small (the fronts are well conditioned)."""
    c = W.lognormal_field(ne, 5)
    pr = _problem(p, ne, s, 0.0, 0.0, c)
    pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=0)
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    b = W.random_rhs(pr.ndof, 1, seed=9)
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    xo = spla.spsolve(Q, b.T).reshape(1, -1)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    assert 1e-10 < err < 1e-3, err
    pr.close()


def test_all_levels_fp64_reproduces_fp64_factor():
    """fp64_levels = tree height and no refinement is the FP64 factorization:
    solves agree bitwise."""
    pr = _problem(3, 32, 8, 0.05, 0.005)
    b = torch.from_numpy(W.random_rhs(pr.ndof, 2, seed=1))
    pr.factor(2.0)
    x64 = pr.solve_q(b).cpu().numpy()
    pr.factor(2.0, "mixed", fp64_levels=pr.info["height"], ir_sweeps=0)
    xm = pr.solve_q(b).cpu().numpy()
    assert np.array_equal(x64, xm)
    assert pr.ir_sweeps() == 0
    pr.factor(2.0)
    assert pr.ir_sweeps() == -1
    pr.close()


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_calibration_history(levels):
    pr = _problem(4, 64, 32, 0.0, 0.0, W.lognormal_field(64, 0))
    hist = pr.factor(5.0, "mixed", fp64_levels=levels, ir_sweeps=-1)
    k = pr.ir_sweeps()
    print("[hist]", levels, k, hist, flush=True)
    assert hist[0] < 1e-3                       # one FP32 solve
    assert hist[1] < 1e-2 * hist[0]             # a sweep gains at least two digits here
    assert 1 <= k <= _riga().RIGA_IR_MAX
    assert hist[k] <= 1e-13
    # the choice rule: the next sweep would gain less than a factor 4 (or the cap)
    assert k == _riga().RIGA_IR_MAX or hist[k + 1] > 0.25 * hist[k]
    for j in range(1, k + 1):
        assert hist[j] <= 0.25 * hist[j - 1]
    # with a residual target: the fewest sweeps reaching it
    for tol in (1e-6, 1e-9, 1e-12):
        h2 = pr.factor(5.0, "mixed", fp64_levels=levels, ir_sweeps=-1, ir_tol=tol)
        k2 = pr.ir_sweeps()
        assert np.array_equal(h2, hist)         # the calibration solve is deterministic
        assert hist[k2] <= tol and (k2 == 0 or hist[k2 - 1] > tol), (tol, k2, hist)
    pr.close()


def test_mixed_apply_op_matches_block_operator():
    p, ne, s, sigma = 3, 32, 8, 2.0
    pr = _problem(p, ne, s, 0.1, 0.01)
    pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=3)
    K, M, C = oasm.assemble(p, ne, s, 0.1, 0.01)
    n = pr.ndof
    v = W.start_block(n, 3, seed=4)
    r = pr.apply_op(torch.from_numpy(v)).cpu().numpy()
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    for q in range(3):
        vu, vl = v[q, :n], v[q, n:]
        ru = -spla.spsolve(Q, sigma * (M @ vu) + C @ vu + M @ vl)
        ref = np.concatenate([ru, sigma * ru + vu])
        assert np.abs(r[q] - ref).max() / np.abs(ref).max() < 1e-11
    pr.close()


def test_mixed_eigs_small_config_closed_form():
    P = W.cfg_small()
    pr = _problem(P.p, P.ne, P.hyper_every, P.alpha, P.beta)
    pr.factor(P.sigma, "mixed", fp64_levels=1, ir_sweeps=-1)
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0)
    assert st == 0 and nconv == P.nev
    ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, P.nev)
    assert (np.abs(lam - ref) / np.abs(ref)).max() <= 1e-10
    assert np.all(eta <= 1e-10)
    pr.close()


def test_mixed_eigs_element_damping_matches_oracle_and_fp64():
    """p=4, s=8 with a lognormal element field (the precision workload's
    ingredients at a size ARPACK handles): the mixed path against the oracle's
    shift-and-invert ARPACK solve and against the FP64 path."""
    p, ne, s, sigma, nev = 4, 32, 8, 5.0, 12
    c = W.lognormal_field(ne, 0)
    pr = _problem(p, ne, s, 0.0, 0.0, c)
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    ref = oeig.shift_invert(K, C, M, sigma, nev)
    pr.factor(sigma)
    lam64, _, eta64, n64, _ = pr.eigs(nev, 2 * nev, block=2, seed=0, vectors=False)
    pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=-1)
    lam, X, eta, nconv, st = pr.eigs(nev, 2 * nev, block=2, seed=0)
    assert st == 0 and nconv == nev and n64 == nev
    # compare up to the cluster ordering at the cut: conjugate pairs / clusters
    assert (np.abs(lam - lam64) / np.abs(lam64)).max() <= 1e-10
    assert (np.abs(lam - ref) / np.abs(ref)).max() <= 1e-10
    assert np.all(eta <= 1e-10)
    U = X.cpu().numpy().T
    norms = (oeig.onenorm(K), oeig.onenorm(C), oeig.onenorm(M))
    for k in range(nev):
        assert oeig.residual(K, C, M, lam[k], U[:, k], norms) <= 1e-10
    pr.close()


def _row_residuals(P, lam, U, rows):
    """|(Q(lam) u)_i| / sum_j |Q(lam)_ij u_j| for sampled rows, every matrix
    entry from the oracle's element-by-element evaluator."""
    n = int(np.sqrt(U.shape[0]))
    out = []
    for i in rows:
        ix, iy = i % n, i // n
        ents = []
        for jy in range(max(0, iy - P.p), min(n, iy + P.p + 1)):
            for jx in range(max(0, ix - P.p), min(n, ix + P.p + 1)):
                j = jy * n + jx
                k, m, c = oasm.entry(P.p, P.ne, P.hyper_every, i, j, P.alpha, P.beta, P.c_elem)
                ents.append((j, k, m, c))
        for q in range(len(lam)):
            l = lam[q]
            terms = np.array([(l * l * m + l * c + k) * U[j, q] for j, k, m, c in ents])
            out.append(abs(terms.sum()) / np.abs(terms).sum())
    return np.array(out)


def test_precision_workload_full_size():
    """The precision workload at its full size (p=4, 1024^2, s=32, 1,252,161
    dofs, lognormal c_e seed 0, sigma 5, 20 pairs): every eigenvalue of the
    mixed path within 1e-10 of the FP64 path, scaled residuals <= 1e-10, and
    sampled rows of Q(lam) u evaluated with the oracle's matrix entries."""
    P = W.cfg_precision()
    pr = _problem(P.p, P.ne, P.hyper_every, 0.0, 0.0, P.c_elem, leaf=16)
    pr.factor(P.sigma)
    lam64, X64, eta64, n64, st64 = pr.eigs(P.nev, P.m, block=2, seed=0)
    print("[full] fp64 done", pr.stats(), flush=True)
    hist = pr.factor(P.sigma, "mixed", fp64_levels=1, ir_sweeps=-1, ir_tol=1e-9)
    k = pr.ir_sweeps()
    lam, X, eta, nconv, st = pr.eigs(P.nev, P.m, block=2, seed=0)
    print("[full] mixed done, sweeps", k, "hist", hist, pr.stats(), flush=True)
    assert st64 == 0 and n64 == P.nev and st == 0 and nconv == P.nev
    rel = np.abs(lam - lam64) / np.abs(lam64)
    for q in range(P.nev):
        print(f"[full] {q:2d} {lam[q]:.12f} rel err vs fp64 {rel[q]:.2e} eta {eta[q]:.1e}", flush=True)
    assert rel.max() <= 1e-10
    assert np.all(eta <= 1e-10) and np.all(eta64 <= 1e-10)
    rng = np.random.default_rng(7)
    rows = rng.choice(pr.ndof, size=6, replace=False)
    pick = [0, 7, 19]
    U = X.cpu().numpy().T[:, pick]
    res = _row_residuals(P, lam[pick], U, rows)
    print("[full] sampled row residuals", res.max(), flush=True)
    assert res.max() <= 1e-8
    pr.close()


def test_stagnated_refinement_falls_back_to_fp64():
    """A refinement target the FP32 factor cannot reach (below the FP64
    residual floor) or a fixed sweep count that misses the caller's target
    gives RIGA_WARN_IR_STAGNATED and leaves an FP64 factor: its solves equal
    those of riga_factor bitwise.  Reachable targets keep the mixed factor."""
    riga = _riga()
    pr = _problem(4, 64, 32, 0.0, 0.0, W.lognormal_field(64, 0))
    b = torch.from_numpy(np.random.default_rng(3).standard_normal((2, pr.ndof)))
    pr.factor(5.0)
    x64 = pr.solve_q(b)
    for sweeps, tol in ((-1, 1e-30), (0, 1e-8), (1, 1e-12)):
        print(f"[case] stagnation sweeps={sweeps} tol={tol}", flush=True)
        pr.factor(5.0, "mixed", fp64_levels=1, ir_sweeps=sweeps, ir_tol=tol)
        assert pr.factor_status == riga.RIGA_WARN_IR_STAGNATED
        assert pr.ir_sweeps() == -1
        assert torch.equal(pr.solve_q(b), x64)
    for sweeps, tol in ((-1, 1e-9), (3, 1e-9), (2, 0.0)):
        pr.factor(5.0, "mixed", fp64_levels=1, ir_sweeps=sweeps, ir_tol=tol)
        assert pr.factor_status == riga.RIGA_OK
        assert pr.ir_sweeps() >= 0
    pr.close()
