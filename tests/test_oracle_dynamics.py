"""Pins of the oracle's implicit-Euler inertia term and ground contact (Sec. 3.1,
Eq. form-full-space-time-integration and Eq. form-reduced-space-time-integration,
with contact as a penalty potential): closed forms of one step of free fall with
and without the ground (no elasticity: every vertex is independent), finite
differences of the reduced gradient and Hessian with both terms active, and the
identity decoder taking the full-space Newton's iterates."""
import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I


def _dyn(p, dt=1.0 / 60, ground=None, k_ground=1e6, young=None):
    q = I.Problem(**{**p.__dict__})
    q.dt = dt
    if young is not None:
        q.young = young
    if ground is not None:
        q.contact_vtx = np.arange(p.nv, dtype=np.int32)
        q.k_ground = k_ground
        q.ground_y = ground
    return q


def test_free_fall_step_closed_form(oracle_mod):
    """Without elasticity the step minimises sum_v m_v (|u_v - qbar_v|^2 / (2 dt^2) - g . u_v):
    u = qbar + dt^2 g on every free vertex."""
    O = oracle_mod
    p = _dyn(I.make_problem("beam", 3, 1, 1, 4, [8], 8, twist=False), young=0.0)
    dt = p.dt
    rng = np.random.default_rng(0)
    qbar = 0.05 * rng.normal(size=(p.nv, 3))
    qbar[p.pinned.astype(bool)] = 0.0
    res = O.Oracle(p).full_newton(p.X.copy(), opts=O.default_opts(rel_tol=1e-12, max_iter=20), qbar=qbar.ravel())
    want = qbar + dt * dt * p.gravity
    free = ~p.pinned.astype(bool)
    assert res["status"] == O.CONVERGED
    assert np.allclose((res["x"] - p.X)[free], want[free], rtol=0, atol=1e-12)


def test_ground_contact_step_closed_form(oracle_mod):
    """With the ground y = y_g: vertices whose free-fall position is below it stop at
    y = (m/dt^2 (y_X + qbar_y + dt^2 g_y) + k y_g) / (m/dt^2 + k); the others fall freely."""
    O = oracle_mod
    base = I.make_problem("beam", 3, 1, 1, 4, [8], 8, twist=False)
    yg = 0.1
    p = _dyn(base, ground=yg, k_ground=1e5, young=0.0)
    dt = p.dt
    o = O.Oracle(p)
    m = o.lumped_mass()
    qbar = np.zeros((p.nv, 3))
    qbar[:, 1] = -0.4 * p.X[:, 0]          # tip side pushed down through the ground
    qbar[p.pinned.astype(bool)] = 0.0
    res = o.full_newton(p.X.copy(), opts=O.default_opts(rel_tol=1e-12, max_iter=50), qbar=qbar.ravel())
    assert res["status"] == O.CONVERGED
    free = ~p.pinned.astype(bool)
    yf = p.X[:, 1] + qbar[:, 1] + dt * dt * p.gravity[1]
    c = m / dt ** 2
    y_want = np.where(yf < yg, (c * yf + p.k_ground * yg) / (c + p.k_ground), yf)
    assert np.any(free & (yf < yg)) and np.any(free & (yf > yg))
    assert np.allclose(res["x"][free, 1], y_want[free], rtol=0, atol=1e-10)


def test_reduced_dynamics_grad_hess_match_differences(oracle_mod):
    O = oracle_mod
    base = I.make_problem("tinyb", 2, 1, 1, 4, [8, 8], 8, bend=True, bias_scale=0.3)
    p = _dyn(base, dt=0.01, ground=-0.02, k_ground=3e4)
    o = O.Oracle(p)
    rng = np.random.default_rng(1)
    z = 0.3 * rng.normal(size=(1, p.r))
    qbar = 0.02 * rng.normal(size=(1, p.n))
    tg, fo = I.loads_for(p, 1)
    E, g, H = o.reduced(z, tg, fo, flags=O.EXACT, qbar=qbar)
    # contact is active at z and the inertia term is not negligible
    x, _ = o.decode(z, want_J=False)
    assert (x[0, :, 1] < p.ground_y).any()
    h = 1e-6
    for k in range(p.r):
        dz = np.zeros_like(z)
        dz[0, k] = h
        Ep, gp, _ = o.reduced(z + dz, tg, fo, flags=O.EXACT, qbar=qbar)
        Em, gm, _ = o.reduced(z - dz, tg, fo, flags=O.EXACT, qbar=qbar)
        assert abs((Ep[0] - Em[0]) / (2 * h) - g[0, k]) <= 1e-6 * np.abs(g).max()
        assert np.allclose((gp[0] - gm[0]) / (2 * h), H[0, :, k], rtol=0, atol=1e-5 * np.abs(H).max())
    # without qbar and contact the terms vanish
    q0 = _dyn(base, dt=0.01)
    E0, g0, _ = O.Oracle(q0).reduced(z, tg, fo, flags=O.EXACT)
    Es, gs, _ = O.Oracle(base).reduced(z, tg, fo, flags=O.EXACT)
    assert np.allclose(E0, Es, rtol=1e-15) and np.allclose(g0, gs, rtol=1e-15)


def test_identity_decoder_dynamics_equals_full_space(oracle_mod):
    """The identity decoder on the free dofs: reduced Newton with inertia and contact
    takes the full-space Newton's iterates (Gauss-Newton on both is exact here)."""
    O = oracle_mod
    base = I.make_problem("beam", 2, 1, 1, 4, [8], 10 ** 9, twist=False)   # every tet, weight 1
    p = _dyn(base, dt=0.02, ground=-0.01, k_ground=2e4)
    free = np.nonzero(np.repeat(~p.pinned.astype(bool), 3))[0]
    p.Ws, p.bs = I.identity_decoder(free, p.n)
    p.r, p.hidden = len(free), []
    rng = np.random.default_rng(2)
    qbar = np.zeros((p.nv, 3))
    qbar[:, 1] = -0.03 * p.X[:, 0]
    qbar[p.pinned.astype(bool)] = 0.0
    o = O.Oracle(p)
    opts = O.default_opts(rel_tol=1e-7, max_iter=50, hess=1)
    red = o.newton(np.zeros((1, p.r)), opts=opts, qbar=qbar.reshape(1, -1))
    full = o.full_newton(p.X.copy(), opts=opts, elem_psd=False, qbar=qbar.ravel())
    assert red["status"][0] == full["status"] == O.CONVERGED
    assert red["iters"][0] == full["iters"]
    u = np.zeros(p.n)
    u[free] = red["z"][0]
    assert np.allclose(u, (full["x"] - p.X).ravel(), rtol=0, atol=1e-10)
    assert abs(red["E"][0] - full["E"]) <= 1e-10 * abs(full["E"])
