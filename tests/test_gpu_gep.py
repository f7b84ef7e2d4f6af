"""The undamped generalized eigenproblem K u = mu M u through the C ABI:
signed factorization with its inertia (Sylvester's law, Sec. 4.1.4) against
the oracle's counts, and spectrum slicing with thick-restart block Lanczos
against the Kronecker-sum closed form (exact in count, every value to 1e-10
relative) and
the dense solver on small meshes.  Every case prints its parameters first."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import assemble as oasm
from oracle import eigen as oeig
from oracle import gep as ogep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _riga():
    from paper_2112_14064_amd import riga
    return riga


def _problem(p, ne, s):
    riga = _riga()
    print(f"[case] gep p={p} ne={ne} s={s}", flush=True)
    pr = riga.Problem(p, ne, s)
    pr.assemble(0.0, 0.0)
    return pr


def _gap_shifts(mu, picks):
    """Midpoints of gaps between distinct eigenvalues (the square has double ones)."""
    gaps = [k for k in range(len(mu) - 1) if mu[k + 1] - mu[k] > 1e-6 * mu[k + 1]]
    return [0.5 * (mu[gaps[i]] + mu[gaps[i] + 1]) for i in picks if i < len(gaps)]


@pytest.mark.parametrize("p,ne,s", [(2, 16, 4), (3, 24, 8), (3, 20, 0), (4, 16, 8)])
def test_inertia_matches_oracle_count(p, ne, s):
    pr = _problem(p, ne, s)
    mu = ogep.gep_closed(p, ne, s, 0.0, np.inf)
    for sh in [0.5 * mu[0]] + _gap_shifts(mu, [0, 3, 10, 30, 60]):
        nu = pr.factor_gep(sh)
        want = ogep.count_below(p, ne, s, sh)
        print(f"  shift {sh:.6g}: nu {nu} oracle {want}", flush=True)
        assert nu == want
    pr.close()


@pytest.mark.parametrize("p,ne,s", [(2, 16, 4), (3, 20, 0)])
def test_signed_solve_matches_sparse_solve(p, ne, s):
    import scipy.sparse.linalg as spla
    pr = _problem(p, ne, s)
    mu = ogep.gep_closed(p, ne, s, 0.0, np.inf)
    sh = _gap_shifts(mu, [12])[0]
    pr.factor_gep(sh)
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    A = (K - sh * M).tocsc()
    b = np.random.default_rng(3).standard_normal((2, pr.ndof))
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    xo = spla.spsolve(A, b.T).T
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"  indefinite solve rel err {err:.3e}", flush=True)
    assert err < 1e-9
    pr.close()


@pytest.mark.parametrize("p,ne,s,lo_i,hi_i,max_slice", [(2, 16, 4, 0, 30, 12), (3, 24, 8, 5, 60, 20),
                                                       (3, 20, 0, 10, 45, 40)])
def test_slices_match_closed_form(p, ne, s, lo_i, hi_i, max_slice):
    pr = _problem(p, ne, s)
    mu_all = ogep.gep_closed(p, ne, s, 0.0, np.inf)
    a = 0.5 * (mu_all[lo_i] + mu_all[lo_i + 1]) if lo_i > 0 else 0.5 * mu_all[0]
    b = _gap_shifts(mu_all, [hi_i])[0]
    want = ogep.gep_closed(p, ne, s, a, b)
    mu, U, eta, count, st, stats = pr.gep_slice(a, b, max_slice=max_slice)
    print(f"  [{a:.4g}, {b:.4g}): count {count} found {len(mu)} oracle {len(want)} status {st} stats {stats}",
          flush=True)
    assert st == 0
    assert count == len(want) == len(mu)
    assert (np.abs(mu - want) / np.abs(want)).max() <= 1e-10
    assert eta.max() <= 1e-10
    # M-orthonormal eigenvectors of the pencil
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    Uh = U.cpu().numpy().T
    G = Uh.T @ (M @ Uh)
    assert np.abs(G - np.eye(len(mu))).max() < 1e-9
    # the scaled residual recomputed with the oracle's matrices and norms
    norms = (oeig.onenorm(K), oeig.onenorm(M))
    eta_o = [ogep.gep_residual(K, M, mu[j], Uh[:, j], norms) for j in range(len(mu))]
    assert max(eta_o) <= 1e-10
    pr.close()


def test_small_mesh_matches_dense_solver():
    p, ne, s = 2, 8, 4
    pr = _problem(p, ne, s)
    K, M, _ = oasm.assemble(p, ne, s, 0.0, 0.0)
    w, _ = ogep.gep_dense(K, M)
    a, b = 0.5 * w[0], _gap_shifts(w, [14])[0]
    mu, U, eta, count, st, stats = pr.gep_slice(a, b, max_slice=8)
    want = w[(w >= a) & (w < b)]
    assert st == 0 and count == len(want) == len(mu)
    assert (np.abs(mu - want) / np.abs(want)).max() <= 1e-10
    pr.close()


@pytest.mark.parametrize("s", [16, 0])
def test_headline_mesh_slices(s):
    """p=3, 256^2, rIGA s=16 (82,369 dofs) and IGA (66,049 dofs): the ~100
    smallest eigenvalues in slices of at most 40, exact in count and every
    value to 1e-10 relative."""
    p, ne = 3, 256
    pr = _problem(p, ne, s)
    mu_all = ogep.gep_closed(p, ne, s, 0.0, 2.5e4)
    b = _gap_shifts(mu_all, [60])[0]
    want = ogep.gep_closed(p, ne, s, 0.0, b)
    mu, U, eta, count, st, stats = pr.gep_slice(0.5 * mu_all[0], b, max_slice=40, vectors=True)
    print(f"  count {count} found {len(mu)} oracle {len(want)} status {st} stats {stats} max eta {eta.max():.2e}",
          flush=True)
    assert st == 0 and count == len(want) == len(mu)
    assert (np.abs(mu - want) / np.abs(want)).max() <= 1e-10
    assert eta.max() <= 1e-10
    pr.close()
