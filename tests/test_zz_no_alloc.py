"""riga_solve_q_noalloc (the solve with the library's static device workspace)
against riga_solve_q on the same factor, through the C ABI: two calls in a
row, the second with a smaller problem, then a mixed factor; the results must
agree bit for bit (same kernels, same launch order) and match SciPy's sparse
solve.  Oversized workspace needs are rejected before any work is queued.
Collected last (a failure here hides no other test); it passes alone in a
fresh process and after the rest of the suite."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble as oasm
from paper_2112_14064_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _riga():
    from paper_2112_14064_amd import riga
    return riga


def _check_case(p, ne, s, sigma, nrhs, mixed=False):
    riga = _riga()
    print(f"[case] noalloc p={p} ne={ne} s={s} sigma={sigma} nrhs={nrhs} mixed={mixed}", flush=True)
    c = W.lognormal_field(ne, 5)
    pr = riga.Problem(p, ne, s)
    pr.assemble(0.05, 0.005, torch.from_numpy(np.ascontiguousarray(c)))
    if mixed:
        pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=4)
    else:
        pr.factor(sigma)
    b_np = W.random_rhs(pr.ndof, nrhs, seed=10 + nrhs)
    b = torch.from_numpy(b_np).to(pr.device).contiguous()
    x_ref = pr.solve_q(b)
    x = torch.full_like(b, float("nan"))
    assert pr.solve_q_noalloc(b, x) == riga.RIGA_OK
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    K, M, C = oasm.assemble(p, ne, s, 0.05, 0.005, c)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    xo = spla.spsolve(Q, b_np.T).reshape(pr.ndof, nrhs).T
    xh = x.cpu().numpy()
    err = np.abs(xh - xo).max() / np.abs(xo).max()
    assert err < 1e-11, err
    pr.close()


def test_noalloc_solve_matches_solve_q_twice_then_smaller():
    _check_case(3, 64, 16, 2.0, 3)
    _check_case(2, 16, 4, 1.0, 1)


def test_noalloc_solve_mixed_factor():
    _check_case(4, 48, 8, 5.0, 2, mixed=True)
    _check_case(2, 12, 4, 1.0, 1, mixed=True)


def test_noalloc_rejects_oversized_workspace_and_unfactored_handle():
    riga = _riga()
    print("[case] noalloc size limit p=4 ne=1024 s=32 (no factor)", flush=True)
    pr = riga.Problem(4, 1024, 32)
    n, u = int(pr.info["ndof"]), int(pr.info["upd_len"])
    limit = 64 << 20
    nrhs_fit = [k for k in range(1, 5) if 8 * k * (n + u) <= limit]
    nrhs_big = [k for k in range(1, 5) if 8 * k * (n + u) > limit]
    assert nrhs_fit and nrhs_big, (n, u)
    for k in nrhs_big:
        b = torch.zeros(k, n, dtype=torch.float64, device=pr.device)
        with pytest.raises(riga.RigaError) as e:
            pr.solve_q_noalloc(b, torch.empty_like(b))
        assert e.value.status == riga.RIGA_ERR_SCRATCH
        assert "RIGA_NOALLOC_SCRATCH_BYTES" in str(e.value)
    b = torch.zeros(nrhs_fit[-1], n, dtype=torch.float64, device=pr.device)
    with pytest.raises(riga.RigaError) as e:   # fits, but nothing is factored yet
        pr.solve_q_noalloc(b, torch.empty_like(b))
    assert e.value.status == riga.RIGA_ERR_STATE
    pr.close()
