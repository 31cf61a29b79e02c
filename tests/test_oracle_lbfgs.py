"""Pins of the oracle's reduced L-BFGS (the paper's main solver, Sec. 5).

The two-loop recursion is checked against the dense BFGS inverse-Hessian
update it stands for (a different formula: explicit r x r products), against
the secant equation, and the solver against the full-space Newton minimum
(an identity decoder makes the reduced problem the full-space one), against
its own exit conditions, and for stationarity under the reduced gradient.
"""
import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I


def _pairs(rng, r, n):
    """(s, y) pairs with positive curvature, y = A s for an SPD A plus noise."""
    M = rng.normal(size=(r, r))
    A = M @ M.T + r * np.eye(r)
    S = rng.normal(size=(n, r))
    Y = S @ A + 0.01 * rng.normal(size=(n, r))
    assert np.all(np.einsum("ij,ij->i", S, Y) > 0)
    return S, Y


def _dense_bfgs(S, Y):
    """H_k from H_0 = gamma I by the BFGS inverse update, oldest pair first."""
    r = S.shape[1]
    gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]) if len(S) else 1.0
    H = gamma * np.eye(r)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        V = np.eye(r) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("r,n", [(1, 1), (5, 3), (16, 10), (7, 7)])
def test_two_loop_matches_dense_bfgs_update(oracle_mod, r, n):
    rng = np.random.default_rng(r * 31 + n)
    S, Y = _pairs(rng, r, n)
    for _ in range(3):
        g = rng.normal(size=r)
        d = oracle_mod.lbfgs_dir(S, Y, g)
        ref = -_dense_bfgs(S, Y) @ g
        assert np.allclose(d, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_two_loop_secant_and_no_pairs(oracle_mod):
    rng = np.random.default_rng(5)
    r = 9
    S, Y = _pairs(rng, r, 4)
    # H_k y_k = s_k for the newest pair
    d = oracle_mod.lbfgs_dir(S, Y, Y[-1])
    assert np.allclose(-d, S[-1], rtol=1e-11, atol=1e-13)
    g = rng.normal(size=r)
    assert np.array_equal(oracle_mod.lbfgs_dir(np.zeros((0, r)), np.zeros((0, r)), g), -g)
    # the direction is a descent direction (H_k is positive definite)
    assert oracle_mod.lbfgs_dir(S, Y, g) @ g < 0


def test_lbfgs_identity_decoder_reaches_full_space_minimum(oracle_mod):
    p = I.make_problem("ident", 2, 1, 1, 1, [], 10 ** 9)
    free = np.nonzero(np.repeat(p.pinned == 0, 3))[0]
    p.Ws, p.bs = I.identity_decoder(free, p.n)
    p.r = len(free)
    o = oracle_mod.Oracle(p)
    t, f = I.loads_for(p, 1, twist_deg=[40.0])
    z = 0.01 * np.random.default_rng(3).normal(size=(1, p.r))
    # 1e-9: near 1e-10 FP64 energy differences stop the Armijo test (exit III)
    lb = o.lbfgs(z, t, f, opts=oracle_mod.default_lbfgs_opts(rel_tol=1e-9))
    assert lb["status"][0] == oracle_mod.CONVERGED
    x, _ = o.decode(z, want_J=False)
    full = o.full_newton(x[0], t[0], None, opts=oracle_mod.default_opts(rel_tol=1e-10, max_iter=60),
                         elem_psd=False)
    xl, _ = o.decode(lb["z"], want_J=False)
    assert full["status"] == oracle_mod.CONVERGED
    assert lb["E"][0] == pytest.approx(full["E"], rel=1e-12)
    assert np.allclose(xl[0], full["x"], rtol=0, atol=1e-7)


def test_lbfgs_c1_converges_stationary(oracle_mod):
    p = I.config("c1")
    o = oracle_mod.Oracle(p)
    z0 = np.vstack([np.zeros(p.r), I.latent_batch(3, p.r)])
    E0, gz0, _ = o.reduced(z0)
    res = o.lbfgs(z0)
    assert np.all(res["status"] == oracle_mod.CONVERGED)
    assert np.all(res["iters"] > 0)
    Es, gs, Hs = o.reduced(res["z"])
    g0 = np.abs(gz0).max(axis=1)
    assert np.all(np.abs(gs).max(axis=1) <= 1e-6 * g0 * (1 + 1e-9))
    assert np.all(res["E"] <= E0)
    assert np.allclose(res["E"], Es, rtol=1e-12)
    # a minimum, not a saddle: the exact reduced Hessian is positive semi-definite there
    for b in range(len(z0)):
        w = np.linalg.eigvalsh(0.5 * (Hs[b] + Hs[b].T))
        assert w.min() > -1e-6 * np.abs(w).max()


def test_lbfgs_forced_exit_statuses(oracle_mod):
    p = I.config("tiny", bias_scale=0.3)
    o = oracle_mod.Oracle(p)
    t, f = I.loads_for(p, 1, twist_deg=[120.0])
    z0 = I.latent_batch(1, p.r)
    r = o.lbfgs(z0, t, f, opts=oracle_mod.default_lbfgs_opts(max_iter=0))
    assert r["status"][0] == oracle_mod.ITER_MAX and r["iters"][0] == 0
    r = o.lbfgs(z0, t, f, opts=oracle_mod.default_lbfgs_opts(ls_max=0))
    assert r["status"][0] == oracle_mod.LS_MAX and r["iters"][0] == 0
    zn = z0.copy(); zn[0, 0] = np.nan
    r = o.lbfgs(zn, t, f)
    assert r["status"][0] == oracle_mod.NONFINITE
    # without history the first step is steepest descent: one iteration with
    # history 0 equals one backtracking step along -g
    r1 = o.lbfgs(z0, t, f, opts=oracle_mod.default_lbfgs_opts(max_iter=1, history=0))
    E, g, _ = o.reduced(z0, t, f)
    alpha = 1.0
    for _ in range(128):
        Et = o.reduced(z0 - alpha * g, t, f, flags=oracle_mod.ENERGY_ONLY)[0][0]
        if Et - E[0] <= 1e-4 * alpha * -(g[0] @ g[0]):
            break
        alpha *= 0.5
    assert np.allclose(r1["z"][0], z0[0] - alpha * g[0], rtol=0, atol=1e-14 * (1 + np.abs(z0).max()))
