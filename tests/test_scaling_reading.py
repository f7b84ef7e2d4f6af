"""The scaling remark of Sec. 6.2.2 (lam = s gamma, C_s = s C, M_s = s^2 M,
s^2 = ||K|| / ||M||) against the B-orthogonal shift-and-invert iteration: the
scaled operator is s R^{-1} S R with R = diag(I, s I), the B-inner product is
invariant under R, and B-orthogonal Arnoldi on both returns the same Ritz
eigenvalues.  CPU only (dense matrices of a small mesh from the oracle)."""
import numpy as np

from oracle import assemble as oasm


def _ops(K, C, M, sigma):
    n = K.shape[0]
    Z, I = np.zeros((n, n)), np.eye(n)
    A = np.block([[Z, I], [-K, -C]])
    B = np.block([[I, Z], [Z, M]])
    return np.linalg.solve(A - sigma * B, B), B


def _arnoldi(S, B, v0, m):
    n = S.shape[0]
    V = np.zeros((n, m + 1)); H = np.zeros((m + 1, m))
    V[:, 0] = v0 / np.sqrt(v0 @ B @ v0)
    for j in range(m):
        w = S @ V[:, j]
        for _ in range(2):
            h = V[:, :j + 1].T @ (B @ w)
            w = w - V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.sqrt(w @ B @ w)
        V[:, j + 1] = w / H[j + 1, j]
    return V, H


def test_scaled_pencil_gives_the_same_iteration():
    K, M, C = oasm.assemble(2, 6, 3, 0.05, 0.005)
    K, M, C = K.toarray(), M.toarray(), C.toarray()
    n = K.shape[0]
    s = np.sqrt(np.abs(K).sum(axis=1).max() / np.abs(M).sum(axis=1).max())
    sigma = 2.0
    S, B = _ops(K, C, M, sigma)
    Ss, Bs = _ops(K, s * C, s * s * M, sigma / s)
    R = np.diag(np.concatenate([np.ones(n), s * np.ones(n)]))
    Ri = np.linalg.inv(R)
    assert np.abs(Ss - s * Ri @ S @ R).max() <= 1e-10 * np.abs(Ss).max()
    x, y = np.random.default_rng(0).standard_normal((2, 2 * n))
    assert abs((Ri @ x) @ Bs @ (Ri @ y) - x @ B @ y) <= 1e-12 * abs(x @ B @ y)
    v0 = np.random.default_rng(1).standard_normal(2 * n)
    m = 12
    V, H = _arnoldi(S, B, v0, m)
    Vs, Hs = _arnoldi(Ss, Bs, Ri @ v0, m)
    assert np.abs(Vs - Ri @ V).max() <= 1e-8 * np.abs(V).max()
    assert np.abs(Hs - s * H).max() <= 1e-8 * s * np.abs(H).max()
    lam = np.sort_complex(sigma + 1.0 / np.linalg.eigvals(H[:m, :m]))
    lam_s = np.sort_complex(s * (sigma / s + 1.0 / np.linalg.eigvals(Hs[:m, :m])))
    assert np.abs(lam - lam_s).max() <= 1e-8 * np.abs(lam).max()
    # planted: the Euclidean inner product is not invariant under R
    assert abs((Ri @ x) @ (Ri @ y) - x @ y) > 1e-3 * abs(x @ y)
