"""Pins of the oracle's PCA basis (the linear subspace baseline): mass
orthonormality, the Eckart-Young residual, optimality against random
subspaces, invariance to a common offset, and exact recovery of snapshots that
lie in a known subspace."""
import numpy as np

from paper_2409_03807_amd import inputs as I


def _setup(oracle_mod, N=40, seed=0):
    p = I.make_problem("blk", 3, 2, 2, 4, [8], 8, bend=True)
    o = oracle_mod.Oracle(p)
    m = np.repeat(o.lumped_mass(), 3)
    rng = np.random.default_rng(seed)
    free = np.repeat(~p.pinned.astype(bool), 3)
    D = rng.normal(size=(N, p.n)) * np.linspace(2.0, 0.1, p.n)   # anisotropic spread
    D[:, ~free] = 0.0
    return p, m, D


def _resid(D, mean, W, m):
    Dc = D - mean
    P = Dc - (Dc * m) @ W @ W.T
    return float(((P ** 2) * m).sum())


def test_pca_basis_is_mass_orthonormal_and_meets_eckart_young(oracle_mod):
    p, m, D = _setup(oracle_mod)
    r = 5
    W, mean, ev = oracle_mod.pca(D, m, r)
    assert np.allclose(W.T @ (W * m[:, None]), np.eye(r), atol=1e-12)
    total = float((((D - mean) ** 2) * m).sum())
    # the residual is the uncaptured sum of squares
    assert abs(_resid(D, mean, W, m) - (total - ev.sum())) <= 1e-10 * total
    assert np.all(np.diff(ev) <= 0)


def test_pca_beats_random_subspaces(oracle_mod):
    p, m, D = _setup(oracle_mod, seed=1)
    r = 4
    W, mean, _ = oracle_mod.pca(D, m, r)
    best = _resid(D, mean, W, m)
    rng = np.random.default_rng(2)
    for _ in range(30):
        Q = rng.normal(size=(p.n, r))
        # mass-orthonormalise
        G = Q.T @ (Q * m[:, None])
        L = np.linalg.cholesky(G)
        Q = Q @ np.linalg.inv(L).T
        assert best <= _resid(D, mean, Q, m) + 1e-9


def test_pca_offset_and_exact_subspace(oracle_mod):
    p, m, D = _setup(oracle_mod, N=30, seed=3)
    r = 3
    W, mean, _ = oracle_mod.pca(D, m, r)
    c = np.random.default_rng(4).normal(size=p.n)
    W2, mean2, _ = oracle_mod.pca(D + c, m, r)
    assert np.allclose(mean2, mean + c, atol=1e-12)
    # same subspace: the mass-inner products of the two bases form an orthogonal matrix
    sv = np.linalg.svd(W.T @ (W2 * m[:, None]), compute_uv=False)
    assert np.allclose(sv, 1.0, atol=1e-10)
    # snapshots inside a known 3-dimensional subspace (plus a mean) are recovered exactly
    rng = np.random.default_rng(5)
    B = rng.normal(size=(p.n, r))
    mu = rng.normal(size=p.n)
    Dk = mu + rng.normal(size=(25, r)) @ B.T
    Wk, mk, evk = oracle_mod.pca(Dk, m, r)
    assert _resid(Dk, mk, Wk, m) <= 1e-20 * float(((Dk - mk) ** 2 * m).sum())
    # the basis spans B's columns: projecting B leaves nothing
    Bc = B - Wk @ (Wk.T @ (B * m[:, None]))
    assert np.linalg.norm(Bc) <= 1e-9 * np.linalg.norm(B)
