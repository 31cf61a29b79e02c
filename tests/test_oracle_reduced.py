"""Pins of the oracle's decoder, reduced objective, Newton solver, full-space
reference and Lipschitz loss.

Every check compares the oracle against something other than itself:
finite differences of a lower-order quantity, the full-space formulation (an
identity decoder turns the reduced problem into the textbook full-space one),
exact scaling laws, invariants of the solver's exit conditions, or brute-force
second differences of the energy.
"""
import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I


def tiny(**kw):
    return I.config("tiny", bias_scale=0.3, **kw)


def fd(fun, z, eps):
    cols = []
    for k in range(len(z)):
        d = np.zeros_like(z); d[k] = eps
        cols.append((fun(z + d) - fun(z - d)) / (2 * eps))
    return np.stack(cols, axis=-1)


# --------------------------------------------------------------------------- decoder
def test_decoder_rest_and_pinned(oracle_mod):
    p = I.config("c1")
    o = oracle_mod.Oracle(p)
    x, J = o.decode(np.zeros((1, p.r)))
    assert np.array_equal(x[0], p.X), "zero-bias decoder maps z=0 to the rest shape"
    z = I.latent_batch(2, p.r)
    x, J = o.decode(z)
    fixed = np.repeat(p.pinned.astype(bool), 3)
    assert np.array_equal(x[:, p.pinned.astype(bool)], np.broadcast_to(p.X[p.pinned.astype(bool)], x[:, p.pinned.astype(bool)].shape))
    assert np.abs(J[:, fixed]).max() == 0.0


def test_decoder_jacobian_and_curvature_fd(oracle_mod):
    p = tiny()
    o = oracle_mod.Oracle(p)
    z = I.latent_batch(1, p.r)[0]
    x, J = o.decode(z[None])
    Jfd = fd(lambda zz: o.decode(zz[None], want_J=False)[0][0].ravel(), z, 1e-6)
    assert np.abs(Jfd - J[0]).max() <= 1e-8 * np.abs(J).max()
    T = o.decode_hess(z)
    Tfd = fd(lambda zz: o.decode(zz[None])[1][0], z, 1e-6)  # (n, r, r)
    assert np.abs(Tfd - T).max() <= 1e-7 * np.abs(T).max()
    assert np.allclose(T, np.swapaxes(T, 1, 2), atol=1e-14)


def test_linear_decoder_has_no_curvature(oracle_mod):
    p = tiny()
    rng = np.random.default_rng(7)
    p.hidden = []
    p.Ws = [rng.normal(scale=0.02, size=(p.n, p.r))]
    p.bs = [np.zeros(p.n)]
    o = oracle_mod.Oracle(p)
    z = I.latent_batch(3, p.r)
    assert np.abs(o.decode_hess(z[0])).max() == 0.0
    t, f = I.loads_for(p, 3)
    Ee, ge, He = o.reduced(z, t, f, flags=oracle_mod.EXACT)
    Eg, gg, Hg = o.reduced(z, t, f, flags=0)
    assert np.array_equal(He, Hg) and np.array_equal(ge, gg)


# --------------------------------------------------------------------------- reduced
@pytest.mark.parametrize("cfg", ["tiny", "c1"])
def test_reduced_gradient_hessian_fd(oracle_mod, cfg):
    p = tiny() if cfg == "tiny" else I.config("c1", bias_scale=0.1)
    o = oracle_mod.Oracle(p)
    t, f = I.loads_for(p, 1, twist_deg=[70.0])
    z = I.latent_batch(1, p.r)[0]
    E, g, H = o.reduced(z[None], t, f)
    Efun = lambda zz: o.reduced(zz[None], t, f, flags=oracle_mod.ENERGY_ONLY)[0][0]
    gfun = lambda zz: o.reduced(zz[None], t, f)[1][0]
    gfd = fd(Efun, z, 1e-6)
    Hfd = fd(gfun, z, 1e-6)
    assert np.abs(gfd - g[0]).max() <= 1e-7 * np.abs(g).max()
    assert np.abs(Hfd - H[0]).max() <= 1e-7 * np.abs(H).max()


def test_all_elements_weight_one_equals_full_energy(oracle_mod):
    p = I.config("c1", bias_scale=0.1)
    o = oracle_mod.Oracle(p)
    z = I.latent_batch(3, p.r)
    E, g, H = o.reduced(z)
    x, _ = o.decode(z, want_J=False)
    for b in range(3):
        Ef, _ = o.full_energy(x[b])
        assert E[b] == pytest.approx(Ef, rel=1e-12)


def test_cubature_weight_scaling(oracle_mod):
    p = tiny()
    p2 = tiny(); p2.cub_w = 2 * p.cub_w
    o, o2 = oracle_mod.Oracle(p), oracle_mod.Oracle(p2)
    z = I.latent_batch(2, p.r)
    fl = oracle_mod.EXACT | oracle_mod.ELASTIC_ONLY
    E1, g1, H1 = o.reduced(z, flags=fl)
    E2, g2, H2 = o2.reduced(z, flags=fl)
    assert np.allclose(E2, 2 * E1, rtol=1e-13)
    assert np.allclose(g2, 2 * g1, rtol=1e-12, atol=1e-12 * np.abs(g1).max())
    assert np.allclose(H2, 2 * H1, rtol=1e-12, atol=1e-12 * np.abs(H1).max())


def identity_problem(oracle_mod):
    """Every tet with weight 1 and a linear decoder selecting the free DOFs."""
    p = I.make_problem("ident", 2, 1, 1, 1, [], 10 ** 9)
    free = np.nonzero(np.repeat(p.pinned == 0, 3))[0]
    p.Ws, p.bs = I.identity_decoder(free, p.n)
    p.r = len(free)
    return p, free


def test_identity_decoder_matches_full_space(oracle_mod):
    p, free = identity_problem(oracle_mod)
    o = oracle_mod.Oracle(p)
    t, f = I.loads_for(p, 1, twist_deg=[40.0])
    rng = np.random.default_rng(3)
    z = 0.01 * rng.normal(size=p.r)
    E, g, H = o.reduced(z[None], t, f)
    x, _ = o.decode(z[None], want_J=False)
    Ef, gf = o.full_energy(x[0], t[0])
    assert E[0] == pytest.approx(Ef, rel=1e-12)
    assert np.allclose(g[0], gf.ravel()[free], rtol=1e-12, atol=1e-9)
    # reduced Newton iterates are the full-space Newton iterates (same policy)
    opts = oracle_mod.default_opts(rel_tol=1e-9, max_iter=60)
    red = o.newton(z[None], t, f, opts=opts)
    full = o.full_newton(x[0], t[0], None, opts=opts, elem_psd=False)
    xr, _ = o.decode(red["z"], want_J=False)
    assert red["status"][0] == oracle_mod.CONVERGED and full["status"] == oracle_mod.CONVERGED
    assert red["iters"][0] == full["iters"]
    assert np.allclose(xr[0], full["x"], rtol=0, atol=1e-9)
    assert red["E"][0] == pytest.approx(full["E"], rel=1e-9)


# --------------------------------------------------------------------------- Newton
def test_newton_c1_converges_and_full_space_reference(oracle_mod):
    p = I.config("c1")
    o = oracle_mod.Oracle(p)
    z0 = np.vstack([np.zeros(p.r), I.latent_batch(3, p.r)])
    E0 = o.reduced(z0, flags=oracle_mod.ENERGY_ONLY)[0]
    res = o.newton(z0)
    assert np.all(res["status"] == oracle_mod.CONVERGED)
    g0 = np.abs(o.reduced(z0)[1]).max(axis=1)
    Es, gs, Hs = o.reduced(res["z"])
    assert np.all(np.abs(gs).max(axis=1) <= 1e-6 * g0 * (1 + 1e-9))
    assert np.all(res["E"] <= E0)
    assert np.allclose(res["E"], Es, rtol=1e-12)
    for b in range(len(z0)):
        w = np.linalg.eigvalsh(0.5 * (Hs[b] + Hs[b].T))
        assert w.min() > -1e-8 * np.abs(w).max()
    # the full-space reference started from q(z*) cannot end above the reduced energy
    x, _ = o.decode(res["z"][:1], want_J=False)
    full = o.full_newton(x[0])
    # FP64 energy differences stop the reference solve's line search near relgrad 1e-7
    assert full["status"] in (oracle_mod.CONVERGED, oracle_mod.LS_MAX)
    assert full["relgrad"] <= 1e-6
    assert full["E"] <= res["E"][0] + 1e-12 * abs(res["E"][0])


def test_newton_forced_exit_statuses(oracle_mod):
    p = tiny()
    o = oracle_mod.Oracle(p)
    t, f = I.loads_for(p, 1, twist_deg=[120.0])
    z0 = I.latent_batch(1, p.r)
    r = o.newton(z0, t, f, opts=oracle_mod.default_opts(max_iter=0))
    assert r["status"][0] == oracle_mod.ITER_MAX and r["iters"][0] == 0
    r = o.newton(z0, t, f, opts=oracle_mod.default_opts(ls_max=0))
    assert r["status"][0] == oracle_mod.LS_MAX
    zn = z0.copy(); zn[0, 0] = np.nan
    r = o.newton(zn, t, f)
    assert r["status"][0] == oracle_mod.NONFINITE
    # an indefinite Hessian without projection is the paper's saddle exit
    rng = np.random.default_rng(11)
    for _ in range(200):
        z = rng.normal(scale=1.5, size=(1, p.r))
        H = o.reduced(z, t, f)[2][0]
        if np.linalg.eigvalsh(0.5 * (H + H.T)).min() < 0:
            break
    else:
        pytest.skip("no indefinite start found")
    r = o.newton(z, t, f, opts=oracle_mod.default_opts(proj=oracle_mod.PROJ_NONE))
    assert r["status"][0] == oracle_mod.NOT_DESCENT and r["iters"][0] == 0
    r = o.newton(z, t, f)
    assert r["status"][0] == oracle_mod.CONVERGED


# --------------------------------------------------------------------------- Lipschitz
def test_lipschitz_basic_properties(oracle_mod):
    p = tiny()
    o = oracle_mod.Oracle(p)
    z1 = I.latent_batch(4, p.r, seed=5)
    z2 = I.latent_batch(4, p.r, seed=6)
    z2[2] = z1[2]
    a = o.lipschitz(z1, z2)
    b = o.lipschitz(z2, z1)
    assert a["n_valid"] == 3 and a["per_pair"][2] == 0.0
    assert np.all(a["per_pair"] >= 0)
    assert np.allclose(a["per_pair"], b["per_pair"], rtol=1e-14)
    assert a["loss"] == pytest.approx(np.delete(a["per_pair"], 2).mean(), rel=1e-14)
    assert a["lip_max"] == pytest.approx(np.sqrt(a["per_pair"].max()), rel=1e-14)


def test_lipschitz_brute_force_second_differences(oracle_mod):
    """Hessians by second differences of the elastic energy alone."""
    p = tiny()
    o = oracle_mod.Oracle(p)
    fl = oracle_mod.ELASTIC_ONLY | oracle_mod.ENERGY_ONLY
    E = lambda z: o.reduced(z[None], flags=fl)[0][0]

    def hess_fd(z, h=1e-3):
        r = len(z)
        H = np.zeros((r, r))
        for i in range(r):
            for j in range(r):
                di = np.zeros(r); di[i] = h
                dj = np.zeros(r); dj[j] = h
                H[i, j] = (E(z + di + dj) - E(z + di - dj) - E(z - di + dj) + E(z - di - dj)) / (4 * h * h)
        return H

    z1 = I.latent_batch(2, p.r, seed=8)
    z2 = I.latent_batch(2, p.r, seed=9)
    res = o.lipschitz(z1, z2)
    for b in range(2):
        dH = hess_fd(z1[b]) - hess_fd(z2[b])
        ell = (dH ** 2).sum() / ((z1[b] - z2[b]) ** 2).sum()
        assert res["per_pair"][b] == pytest.approx(ell, rel=1e-4)
