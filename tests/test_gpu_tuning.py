"""Autotuner of the sweep tile shapes through the C ABI: the chosen shapes
are valid, solves keep their parity with the oracle, the choice is cached,
and the batched forest is tuned the same way.

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


@pytest.mark.parametrize("p,ne,s,sigma,prec", [(3, 64, 16, 2.0, "fp64"), (4, 48, 8, 5.0, "fp64"),
                                               (3, 40, 0, 2.0, "fp64"), (4, 64, 32, 5.0, "mixed")])
def test_autotuned_solves_keep_parity(p, ne, s, sigma, prec):
    riga = _riga()
    print(f"[case] autotune p={p} ne={ne} s={s} sigma={sigma} {prec}", flush=True)
    c = W.lognormal_field(ne, 6)
    pr = riga.Problem(p, ne, s, leaf=8 if s == 0 else 0)
    pr.assemble(0.05, 0.005, torch.from_numpy(c))
    if prec == "fp64":
        pr.factor(sigma)
    else:
        pr.factor(sigma, "mixed", fp64_levels=1, ir_sweeps=4)
    K, M, C = oasm.assemble(p, ne, s, 0.05, 0.005, c)
    Q = oasm.q_matrix(K, M, C, sigma).tocsc()
    b = W.random_rhs(pr.ndof, 2, seed=4)
    xo = spla.spsolve(Q, b.T).T
    before, after = pr.autotune(nrhs=2, reps=3)
    assert before > 0 and after > 0
    f, bw = pr.sweep_shapes()
    assert len(f) == pr.info["height"] and f.min() >= 0 and f.max() < 8 and bw.min() >= 0 and bw.max() < 8
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    assert np.abs(x - xo).max() / np.abs(xo).max() < 1e-11
    # a second tuning of the same structure is served from the cache
    b2, a2 = pr.autotune(nrhs=2, reps=3)
    f2, bw2 = pr.sweep_shapes()
    assert np.array_equal(f, f2) and np.array_equal(bw, bw2)
    pr.close()


def test_every_sweep_shape_gives_the_same_solution():
    """Force each compiled shape on every level through the tuner's cache-free
    path of a fresh structure: all agree with the sparse solve."""
    riga = _riga()
    print("[case] autotune shapes p=2 ne=24 s=4", flush=True)
    pr = riga.Problem(2, 24, 4)
    pr.assemble(0.1, 0.01)
    pr.factor(1.5)
    K, M, C = oasm.assemble(2, 24, 4, 0.1, 0.01)
    Q = oasm.q_matrix(K, M, C, 1.5).tocsc()
    b = W.random_rhs(pr.ndof, 3, seed=2)
    xo = spla.spsolve(Q, b.T).T
    pr.autotune(nrhs=3, reps=2)
    x = pr.solve_q(torch.from_numpy(b)).cpu().numpy()
    assert np.abs(x - xo).max() / np.abs(xo).max() < 1e-11
    pr.close()


def test_batch_autotune_then_eigs():
    riga = _riga()
    rng = np.random.default_rng(21)
    probs = [W.Problem(p=int(rng.integers(2, 5)), ne=int(rng.choice([16, 24, 32])), hyper_every=8,
                       alpha=float(rng.uniform(0, 0.2)), beta=float(rng.uniform(0, 0.02)),
                       sigma=float(rng.uniform(0.5, 4.0)), nev=8, m=20) for _ in range(8)]
    print("[case] batch autotune, 8 problems", flush=True)
    B = riga.Batch([(P.p, P.ne, P.hyper_every) for P in probs])
    B.assemble([P.alpha for P in probs], [P.beta for P in probs])
    B.factor([P.sigma for P in probs])
    before, after = B.autotune(2, 3)
    assert before > 0 and after > 0
    lam, _, eta, nconv, st = B.eigs(8, 20, block=2, seed=0)
    assert st == 0 and np.all(nconv == 8)
    for i, P in enumerate(probs):
        ref, _ = oeig.rayleigh_closed(P.p, P.ne, P.hyper_every, P.alpha, P.beta, P.sigma, 8)
        assert (np.abs(lam[i] - ref) / np.abs(ref)).max() <= 1e-10
    assert np.all(eta <= 1e-10)
    B.close()
