"""Pins of the CPU oracle against values fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself: numbers the
paper prints, closed forms, invariants, or independent routes (dense QZ vs
closed form vs ARPACK).  All run on the CPU.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import assemble as oasm
from oracle import bspline as obs
from oracle import eigen as oeig
from oracle import space as ospace

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --- space construction -------------------------------------------------------

def test_fig_matpatterns_counts():
    """N and nnz of the 64x64, p=4 H(curl) IGA and rIGA matrices (fig. MatPatterns)."""
    g = _gold("fig_matpatterns.json")
    assert ospace.hcurl_counts(g["p"], g["ne"], 0) == (g["iga"]["N"], g["iga"]["nnz"])
    assert ospace.hcurl_counts(g["p"], g["ne"], g["macro"]) == (g["riga"]["N"], g["riga"]["nnz"])


def test_scalar_dimensions():
    # 16x16, p=2, C^0 every 4: 19 functions per direction after Dirichlet
    assert ospace.scalar_counts(2, 16, 4)[0] == 361
    # rIGA adds (p-1) functions per hyperplane per direction (Sec. 3.3)
    for p, ne, s in [(3, 256, 16), (4, 1024, 32), (3, 512, 16), (2, 48, 8)]:
        n_iga = ospace.n1d_dirichlet(p, ne, 0)
        n_riga = ospace.n1d_dirichlet(p, ne, s)
        assert n_iga == ne + p - 2
        assert n_riga - n_iga == (ne // s - 1) * (p - 1)
    # rIGA has more dofs and more nonzeros than IGA (Sec. 3.3)
    n_i, z_i = ospace.scalar_counts(3, 64, 0)
    n_r, z_r = ospace.scalar_counts(3, 64, 16)
    assert n_r > n_i and z_r > z_i


# --- B-spline basis -------------------------------------------------------------

@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 12, 4), (4, 16, 8), (3, 10, 0)])
def test_partition_of_unity(p, ne, s):
    kv = obs.knot_vector(p, ne, s)
    x = np.random.default_rng(1).uniform(0, 1, 200)
    B = obs.basis(kv, p, x)
    D = obs.basis_deriv(kv, p, x)
    assert np.all(B >= -1e-15)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-10)


def test_c0_at_hyperplane():
    """At a knot of multiplicity p exactly one function is nonzero (C^0)."""
    p, ne, s = 3, 8, 4
    kv = obs.knot_vector(p, ne, s)
    B = obs.basis(kv, p, np.array([0.5]))
    assert np.count_nonzero(np.abs(B) > 1e-15) == 1
    assert abs(B.max() - 1.0) < 1e-15


def test_derivative_matches_finite_difference():
    p, ne, s = 3, 6, 3
    kv = obs.knot_vector(p, ne, s)
    x = np.array([0.13, 0.41, 0.77])
    h = 1e-6
    fd = (obs.basis(kv, p, x + h) - obs.basis(kv, p, x - h)) / (2 * h)
    assert np.allclose(obs.basis_deriv(kv, p, x), fd, atol=1e-7)


# --- assembly -------------------------------------------------------------------

def _cardinal(n, x, deriv=0):
    """Cardinal B-spline of degree n on [0, n+1] by the truncated-power formula,
    in exact rational arithmetic."""
    x = Fraction(x)
    tot = Fraction(0)
    for k in range(n + 2):
        t = x - k
        if t > 0:
            pw = n - deriv
            coef = math.perm(n, deriv)
            tot += (-1) ** k * math.comb(n + 1, k) * coef * t ** pw
    return tot / math.factorial(n)


@pytest.mark.parametrize("p", [2, 3])
def test_interior_rows_are_cardinal_bsplines(p):
    g = _gold("cardinal_bspline.json")
    ne = 24
    h = 1.0 / ne
    K1, M1 = oasm.assemble_1d(p, ne, 0)
    row = M1.shape[0] // 2
    exact_m = [_cardinal(2 * p + 1, p + 1 + k) for k in range(-p, p + 1)]
    gold = g["mass"][str(p)]
    assert [Fraction(a, gold["den"]) for a in gold["num"]] == exact_m
    assert np.allclose(M1[row, row - p:row + p + 1] / h, [float(v) for v in exact_m], rtol=1e-13)
    exact_k = [-_cardinal(2 * p + 1, p + 1 + k, deriv=2) for k in range(-p, p + 1)]
    assert np.allclose(K1[row, row - p:row + p + 1] * h, [float(v) for v in exact_k], rtol=1e-12)
    if p == 2:
        gk = g["stiffness_p2"]
        assert [Fraction(a, gk["den"]) for a in gk["num"]] == exact_k
    # entries beyond the band vanish
    assert np.all(M1[row, :row - p] == 0) and np.all(M1[row, row + p + 1:] == 0)


@pytest.mark.parametrize("p,ne,s", [(2, 8, 4), (3, 8, 4), (3, 8, 0)])
def test_area_and_constant_kernel(p, ne, s):
    """Partition of unity in 2-D: sum of all mass entries = area 1 and the
    stiffness annihilates the constant (no Dirichlet elimination)."""
    K1, M1 = oasm.assemble_full_nodirichlet(p, ne, s)
    M2 = np.kron(M1, M1)
    assert abs(M2.sum() - 1.0) < 1e-13
    assert abs(M1.sum() - 1.0) < 1e-14
    assert np.abs(K1.sum(axis=1)).max() < 1e-11


@pytest.mark.parametrize("p,ne,s", [(2, 16, 4), (3, 12, 4), (4, 10, 5), (3, 9, 0)])
def test_kronecker_identity(p, ne, s):
    """2-D element-by-element Gauss assembly equals the Kronecker form built
    from the 1-D matrices (the tensor rule factorises on the identity map)."""
    K, M, C = oasm.assemble(p, ne, s, 0.3, 0.02)
    K1, M1 = oasm.assemble_1d(p, ne, s)
    Kk = np.kron(M1, K1) + np.kron(K1, M1)
    Mk = np.kron(M1, M1)
    assert np.abs(K.toarray() - Kk).max() < 1e-12 * np.abs(Kk).max()
    assert np.abs(M.toarray() - Mk).max() < 1e-14 * np.abs(Mk).max() + 1e-18
    assert np.abs(C.toarray() - (0.3 * Mk + 0.02 * Kk)).max() < 1e-12


def test_entry_by_entry_matches_assembly():
    p, ne, s = 3, 8, 4
    c = np.random.default_rng(5).lognormal(-3, 0.5, (ne, ne))
    K, M, C = oasm.assemble(p, ne, s, 0.1, 0.01, c)
    rng = np.random.default_rng(3)
    rows, cols = K.nonzero()
    for t in rng.choice(len(rows), 25, replace=False):
        a, b = rows[t], cols[t]
        k, m, cc = oasm.entry(p, ne, s, a, b, 0.1, 0.01, c)
        assert abs(k - K[a, b]) < 1e-13 * max(1, abs(k))
        assert abs(m - M[a, b]) < 1e-16 + 1e-13 * abs(m)
        assert abs(cc - C[a, b]) < 1e-13 * max(1e-3, abs(cc))


def test_element_damping_uniform_equals_rayleigh():
    p, ne, s = 2, 8, 4
    K, M, C1 = oasm.assemble(p, ne, s, 0.0, 0.0, np.full((ne, ne), 0.07))
    _, _, C2 = oasm.assemble(p, ne, s, 0.07, 0.0)
    assert abs(C1 - C2).max() < 1e-15


def test_spd_and_structure():
    K, M, C = oasm.assemble(2, 8, 4, 0.1, 0.01)
    for A in (K, M, C):
        assert abs(A - A.T).max() < 1e-15
    assert np.linalg.eigvalsh(M.toarray()).min() > 0
    Q = oasm.q_matrix(K, M, C, 1.5).toarray()
    assert np.linalg.eigvalsh(Q).min() > 0


# --- spectrum ----------------------------------------------------------------------

def test_three_routes_agree_small_config():
    """Dense QZ on the companion pencil, the Rayleigh closed form and ARPACK
    shift-and-invert give the same 10 (+4) eigenvalues nearest sigma."""
    p, ne, s, a, b, sg, nev = 2, 16, 4, 0.1, 0.01, 1.0, 14
    K, M, C = oasm.assemble(p, ne, s, a, b)
    lam_d, _ = oeig.dense_qep(K, C, M)
    ld = oeig.nearest(lam_d, sg, nev)
    lc, mu = oeig.rayleigh_closed(p, ne, s, a, b, sg, nev)
    ls = oeig.shift_invert(K, C, M, sg, nev)
    assert np.abs(ld - lc).max() < 1e-12 * np.abs(lc).max()
    assert np.abs(ls - lc).max() < 1e-12 * np.abs(lc).max()
    # the quadratic relation with mu holds for every returned value
    assert np.abs(lc ** 2 + (a + b * mu) * lc + mu).max() < 1e-10 * mu.max()
    # Re lam < 0 and conjugate pairs (Sec. 2.2: K, C PSD, M PD)
    assert np.all(lc.real < 0)
    l12 = lc[:12]  # ranks 13-14 cut a 4-fold cluster: check closure below the cut
    assert np.allclose(np.sort_complex(l12), np.sort_complex(np.conj(l12)))


def test_cluster_straddles_cutoff():
    """Ranks 9..12 of the small configuration are the 4-fold cluster
    mu_13 = mu_31 (two conjugate pairs of a double eigenvalue)."""
    lc, mu = oeig.rayleigh_closed(2, 16, 4, 0.1, 0.01, 1.0, 12)
    assert np.allclose(mu[8:12], mu[8], rtol=1e-12)
    assert abs(mu[7] - mu[8]) > 1e-3 * mu[8]
    assert mu[8] / np.pi ** 2 == pytest.approx(10.0, rel=1e-3)


def test_analytic_spectrum_limit():
    """mu_h -> pi^2 (i^2 + j^2) (Sec. 6.4.1) with the optimal rate h^(2p)."""
    g = _gold("analytic_spectrum.json")
    assert round(np.pi ** 2 * (g["i"] ** 2 + g["j"] ** 2), g["printed_digits"]) == g["lambda"]
    p = 2
    errs = []
    for ne in (8, 16, 32):
        mu = oeig.generalized_mu(p, ne, 0, 1)[0]
        errs.append(mu / (2 * np.pi ** 2) - 1)
    assert errs[0] > errs[1] > errs[2] > 0
    rate = np.log2(errs[1] / errs[2])
    assert 2 * p - 0.3 < rate < 2 * p + 0.5


def test_rayleigh_ritz_riga_below_iga():
    """S_IGA is a subspace of S_rIGA (raising knot multiplicity enlarges the
    spline space), so index-wise mu_exact <= mu_rIGA <= mu_IGA."""
    for p, ne, s in [(2, 16, 4), (3, 32, 16), (4, 16, 8)]:
        cnt = 30
        mr = oeig.generalized_mu(p, ne, s, cnt)
        mi = oeig.generalized_mu(p, ne, 0, cnt)
        ij = sorted(i * i + j * j for i in range(1, 12) for j in range(1, 12))[:cnt]
        exact = np.pi ** 2 * np.array(ij, dtype=float)
        assert np.all(mr <= mi * (1 + 1e-13))
        assert np.all(exact <= mr * (1 + 1e-13))


def test_closed_form_matches_sparse_generalized():
    """The 1-D Kronecker route for mu agrees with a sparse 2-D generalized
    eigensolve on the assembled K, M."""
    import scipy.sparse.linalg as spla
    p, ne, s = 3, 16, 8
    K, M, C = oasm.assemble(p, ne, s)
    w = np.sort(spla.eigsh(K.tocsc(), k=8, M=M.tocsc(), sigma=0.0, which="LM")[0])
    mu = oeig.generalized_mu(p, ne, s, 8)
    assert np.allclose(w, mu, rtol=1e-11)


def test_residual_small_for_true_pairs_and_large_otherwise():
    K, M, C = oasm.assemble(2, 8, 4, 0.1, 0.01)
    lam, U = oeig.dense_qep(K, C, M)
    o = oeig.canonical_order(lam, 1.0)[:6]
    for k in o:
        assert oeig.residual(K, C, M, lam[k], U[:, k]) < 1e-13
    assert oeig.residual(K, C, M, lam[o[0]] * (1 + 1e-6), U[:, o[0]]) > 1e-9


def test_canonical_order():
    lam = np.array([1 + 2j, 1 - 2j, 0.5 + 0j, 1 + 2j * (1 + 1e-12), 3 + 0j])
    o = oeig.canonical_order(lam, 1.0)
    # |lam-1|: 2, 2, 0.5, 2(1+1e-12), 2 -> 0.5 first, then the 2-cluster by Im desc
    assert o[0] == 2
    assert list(o[1:3]) in ([3, 0], [0, 3])
    assert set(o[3:]) == {1, 4}
    assert lam[o[3]].imag >= lam[o[4]].imag


# --- adjoint -----------------------------------------------------------------------

def test_adjoint_uniform_closed_form():
    """For C = c M, lam^2 + c lam + mu = 0 gives d lam/dc = -lam/(2 lam + c);
    since sum_e M_e = M the element sensitivities sum to it."""
    p, ne, s, c = 2, 8, 4, 0.3
    K, M, C = oasm.assemble(p, ne, s, c, 0.0)
    lam, U = oeig.dense_qep(K, C, M)
    o = oeig.canonical_order(lam, 1.0)[:6]
    d = oadj.dlam_dc(p, ne, s, M, C, lam[o], U[:, o])
    assert np.allclose(d.sum(axis=(1, 2)), -lam[o] / (2 * lam[o] + c), rtol=1e-10)


def test_adjoint_matches_central_differences():
    p, ne, s, sg, nev = 2, 8, 4, 1.0, 4
    c = np.random.default_rng(7).lognormal(-3, 0.5, (ne, ne))
    K, M, C = oasm.assemble(p, ne, s, 0.0, 0.0, c)
    lam, U = oeig.dense_qep(K, C, M)
    o = oeig.canonical_order(lam, sg)[:nev]
    g = oadj.grad_sum_re(p, ne, s, M, C, lam[o], U[:, o])

    def L(cc):
        K2, M2, C2 = oasm.assemble(p, ne, s, 0.0, 0.0, cc)
        return oeig.nearest(oeig.dense_qep(K2, C2, M2)[0], sg, nev).real.sum()

    # dense QZ carries ~1e-14 |lam| noise, so h = 1e-4 keeps the roundoff
    # floor (~1e-9) and the O(h^2) truncation (~1e-8) far below the check
    h = 1e-4
    for e in [(0, 0), (3, 5), (7, 2)]:
        cp, cm = c.copy(), c.copy()
        cp[e] += h
        cm[e] -= h
        fd = (L(cp) - L(cm)) / (2 * h)
        assert abs(g[e] - fd) < 1e-4 * abs(fd) + 1e-8


# --- planted mistakes: the pins above must catch plausible oracle errors -------------

def test_pins_catch_dropped_damping_term(monkeypatch):
    """A closed form that forgets beta*mu disagrees with dense QZ."""
    p, ne, s, a, b, sg, nev = 2, 16, 4, 0.1, 0.01, 1.0, 10
    K, M, C = oasm.assemble(p, ne, s, a, b)
    ld = oeig.nearest(oeig.dense_qep(K, C, M)[0], sg, nev)
    lc_bad, _ = oeig.rayleigh_closed(p, ne, s, a, 0.0, sg, nev)
    assert np.abs(ld - lc_bad).max() > 1e-4


def test_pins_catch_wrong_multiplicity():
    """A hyperplane multiplicity p-2 instead of p-1 breaks the fig. MatPatterns pin."""
    def counts_bad(p, ne, macro):
        ku = obs.knot_vector(p - 1, ne, macro, mult=p - 2)
        kv = obs.knot_vector(p, ne, macro, mult=p - 2)
        su, sv = ospace.supports(ku, p - 1), ospace.supports(kv, p)
        return 2 * len(su) * len(sv)
    g = _gold("fig_matpatterns.json")
    assert counts_bad(g["p"], g["ne"], g["macro"]) != g["riga"]["N"]


def test_pins_catch_transposed_derivative_sign():
    """Flipping the sign of one derivative term breaks the FD derivative pin."""
    p, ne = 3, 6
    kv = obs.knot_vector(p, ne, 3)
    x = np.array([0.13, 0.41, 0.77])
    Nm = obs.basis(kv, p - 1, x)
    n = obs.n_functions(kv, p)
    bad = np.zeros((3, n))
    for i in range(n):
        d1, d2 = kv[i + p] - kv[i], kv[i + p + 1] - kv[i + 1]
        if d1 > 0:
            bad[:, i] += p / d1 * Nm[:, i]
        if d2 > 0:
            bad[:, i] += p / d2 * Nm[:, i + 1]     # wrong sign
    h = 1e-6
    fd = (obs.basis(kv, p, x + h) - obs.basis(kv, p, x - h)) / (2 * h)
    assert not np.allclose(bad, fd, atol=1e-3)


# --- element mass, Q(lambda) and the scaled residual ---------------------------------

def _scatter_element_masses(p, ne, s, elem_fn):
    """sum_e M_e scattered to the Dirichlet dofs, with M_e from elem_fn."""
    N = ospace.scalar_counts(p, ne, s)[0]
    out = np.zeros((N, N))
    for ey in range(ne):
        for ex in range(ne):
            dofs, Me = elem_fn(p, ne, s, ex, ey)
            ok = np.flatnonzero((dofs >= 0) & (dofs < N))
            out[np.ix_(dofs[ok], dofs[ok])] += Me[np.ix_(ok, ok)]
    return out


def _element_mass_swapped_xy(p, ne, s, ex, ey):
    """Planted mistake: the y factor of the tensor basis taken from element ex."""
    kv, first, B, D, w = oasm._element_tables(p, ne, s)
    n1 = obs.n_functions(kv, p) - 2
    nl = p + 1
    Phi = np.einsum("yb,xa->yxba", B[ex], B[ey]).reshape(nl * nl, nl * nl)
    Me = np.einsum("q,qa,qb->ab", np.outer(w, w).reshape(-1), Phi, Phi)
    dofs = [(first[ey] + ly - 1) * n1 + (first[ex] + lx - 1)
            if (1 <= first[ex] + lx <= n1 and 1 <= first[ey] + ly <= n1) else -1
            for ly in range(nl) for lx in range(nl)]
    return np.array(dofs), Me


def _element_mass_no_dirichlet_mask(p, ne, s, ex, ey):
    """Planted mistake: boundary functions are not dropped from the dof map."""
    dofs, Me = oasm.element_mass_2d(p, ne, s, ex, ey)
    kv, first, B, D, w = oasm._element_tables(p, ne, s)
    n1 = obs.n_functions(kv, p) - 2
    nl = p + 1
    bad = np.array([(first[ey] + ly - 1) * n1 + (first[ex] + lx - 1) for ly in range(nl) for lx in range(nl)])
    return bad, Me


@pytest.mark.parametrize("p,ne,s", [(3, 8, 4), (2, 6, 0), (4, 8, 4)])
def test_element_mass_2d_scatters_to_assembled_mass(p, ne, s):
    """sum_e M_e = M (the mass form is additive over elements, Sec. 3.1): the
    element matrices of element_mass_2d, scattered to their dofs, rebuild the
    assembled M; and u^T M_e u agrees with the 1-D Kronecker route of the
    adjoint's element forms (M_e = M1_ey (x) M1_ex on the tensor basis)."""
    _, M, _ = oasm.assemble(p, ne, s)
    Md = M.toarray()
    S = _scatter_element_masses(p, ne, s, oasm.element_mass_2d)
    assert np.abs(S - Md).max() <= 1e-15 * np.abs(Md).max()
    u = np.random.default_rng(11).standard_normal(M.shape[0])
    q = oadj.element_quadratic_forms(p, ne, s, u)[0]
    for ex, ey in [(0, 0), (ne - 1, 1), (ne // 2, ne // 2 - 1), (1, ne - 1)]:
        dofs, Me = oasm.element_mass_2d(p, ne, s, ex, ey)
        ok = dofs >= 0
        ue = u[dofs[ok]]
        assert abs(ue @ Me[np.ix_(ok, ok)] @ ue - q[ey, ex]) <= 1e-14 * abs(q[ey, ex]) + 1e-18


@pytest.mark.parametrize("bad", [_element_mass_swapped_xy, _element_mass_no_dirichlet_mask])
def test_pins_catch_element_mass_mistakes(bad):
    """A swapped tensor factor (elements differ in x and y near the
    hyperplanes and the boundary) or a missing Dirichlet mask breaks the
    scatter pin."""
    p, ne, s = 3, 8, 4
    Md = oasm.assemble(p, ne, s)[1].toarray()
    S = _scatter_element_masses(p, ne, s, bad)
    assert np.abs(S - Md).max() > 1e-6 * np.abs(Md).max()


def test_q_matrix_annihilates_qz_eigenvectors():
    """Q(lam) u = 0 for eigenpairs of the companion pencil (eq. QuadEig /
    eq. Linearization), at complex lam: q_matrix is lam^2 M + lam C + K."""
    K, M, C = oasm.assemble(2, 8, 4, 0.1, 0.01, np.random.default_rng(4).lognormal(-3, 0.5, (8, 8)))
    lam, U = oeig.dense_qep(K, C, M)
    scale = oeig.onenorm(K)
    for k in oeig.canonical_order(lam, 1.0)[:8]:
        assert abs(lam[k].imag) > 0.1
        r = oasm.q_matrix(K, M, C, lam[k]) @ U[:, k]
        assert np.linalg.norm(r) <= 1e-11 * scale * np.linalg.norm(U[:, k])


def test_pins_catch_q_matrix_mistakes():
    """sigma M for sigma^2 M, or C and M exchanged, leave a large residual."""
    K, M, C = oasm.assemble(2, 8, 4, 0.1, 0.01)
    lam, U = oeig.dense_qep(K, C, M)
    k = oeig.canonical_order(lam, 1.0)[0]
    u = U[:, k]
    scale = oeig.onenorm(K) * np.linalg.norm(u)
    for bad in (lam[k] * M + lam[k] * C + K, lam[k] ** 2 * C + lam[k] * M + K):
        assert np.linalg.norm(bad @ u) > 1e-4 * scale


_ETA_K = np.array([[4.0, 0.0], [3.0, 9.0]])    # column sums 7, 9; row sums 4, 12
_ETA_C = np.array([[1.0, 2.0], [0.0, 0.5]])    # column sums 1, 2.5
_ETA_M = np.array([[1.0, 0.0], [1.0, 2.0]])    # column sums 2, 2; row sums 1, 3
_ETA_LAM = 1.0 + 1.0j
_ETA_U = np.array([1.0, 1.0])


def test_residual_hand_computed():
    """eta for 2 x 2 coefficients worked by hand: lam = 1 + i, lam^2 = 2i,
    Q(lam) u = K u + lam C u + lam^2 M u = [4 + 3 (1+i) + 2i, 12 + 0.5 (1+i) + 6i]
    = [7 + 5i, 12.5 + 6.5i]; ||Q u||_2 = sqrt(49 + 25 + 156.25 + 42.25) = sqrt(272.5);
    |lam|^2 ||M||_1 + |lam| ||C||_1 + ||K||_1 = 2*2 + sqrt(2)*2.5 + 9; ||u||_2 = sqrt(2)."""
    eta = oeig.residual(_ETA_K, _ETA_C, _ETA_M, _ETA_LAM, _ETA_U)
    want = math.sqrt(272.5) / ((4.0 + 2.5 * math.sqrt(2.0) + 9.0) * math.sqrt(2.0))
    assert eta == pytest.approx(want, rel=1e-15)


def test_pins_catch_residual_normalisation_mistakes():
    """A dropped |lam|^2, the infinity norm or an unnormalised u give other values."""
    want = math.sqrt(272.5) / ((4.0 + 2.5 * math.sqrt(2.0) + 9.0) * math.sqrt(2.0))
    num = math.sqrt(272.5)
    bads = [
        num / ((2.0 * 2.0 ** 0.5 + 2.5 * math.sqrt(2.0) + 9.0) * math.sqrt(2.0)),   # |lam| for |lam|^2
        num / ((2.0 * 3.0 + math.sqrt(2.0) * 3.0 + 12.0) * math.sqrt(2.0)),         # infinity norms
        num / (4.0 + 2.5 * math.sqrt(2.0) + 9.0),                                   # ||u|| dropped
    ]
    for b in bads:
        assert abs(b - want) > 1e-3 * want
    # and the oracle's own value is not any of them
    eta = oeig.residual(_ETA_K, _ETA_C, _ETA_M, _ETA_LAM, _ETA_U)
    assert all(abs(eta - b) > 1e-3 * want for b in bads)
