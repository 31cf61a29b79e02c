"""Pins of the oracle's stable Neo-Hookean density and tetrahedron element
(the material the paper cites for its supervised examples, Sec. 5.1).

The paper gives no formula, so the pins are closed forms and invariants:
rest state, frame invariance, uniaxial stretch, the linear-elastic limit with
the configured (E, nu), and finite differences of energy -> stress -> tangent.
"""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
MU, LAM_L, LAM = GOLD["mu"], GOLD["lambda_lame"], GOLD["lambda_snh"]


def rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_lame_reading(oracle_mod):
    mu, lam = oracle_mod.lame(1e5, 0.45)
    assert mu == pytest.approx(MU, rel=1e-14)
    assert lam == pytest.approx(LAM, rel=1e-14)


def test_rest_state_zero(oracle_mod):
    I3 = np.eye(3)
    assert oracle_mod.psi(I3, MU, LAM) == 0.0
    assert np.abs(oracle_mod.pk1(I3, MU, LAM)).max() == 0.0


def test_frame_invariance(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(5):
        F = np.eye(3) + 0.4 * rng.normal(size=(3, 3))
        R = rot(rng)
        assert oracle_mod.psi(R @ F, MU, LAM) == pytest.approx(oracle_mod.psi(F, MU, LAM), rel=1e-13)
        assert np.allclose(oracle_mod.pk1(R @ F, MU, LAM), R @ oracle_mod.pk1(F, MU, LAM), rtol=1e-12, atol=1e-9)


def test_uniaxial_closed_form(oracle_mod):
    for s in [0.5, 0.9, 1.3, 2.0, -0.4]:
        F = np.diag([s, 1.0, 1.0])
        want = MU / 2 * (s * s - 1) - MU * (s - 1) + LAM / 2 * (s - 1) ** 2
        assert oracle_mod.psi(F, MU, LAM) == pytest.approx(want, rel=1e-13, abs=1e-9)


def test_linearisation_is_isotropic_linear_elasticity(oracle_mod):
    """d2psi/dF2 at F = I equals mu (d_ik d_jl + d_il d_jk) + lambda_Lame d_ij d_kl."""
    A = oracle_mod.dpdf(np.eye(3), MU, LAM)
    d = np.eye(3)
    want = np.zeros((9, 9))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    want[3 * j + i, 3 * l + k] = (MU * (d[i, k] * d[j, l] + d[i, l] * d[j, k])
                                                  + LAM_L * d[i, j] * d[k, l])
    assert np.allclose(A, want, rtol=1e-12, atol=1e-6)


def test_stress_and_tangent_by_finite_differences(oracle_mod):
    rng = np.random.default_rng(1)
    for F0 in [np.eye(3) + 0.3 * rng.normal(size=(3, 3)), np.diag([0.7, 1.2, -0.5])]:
        P = oracle_mod.pk1(F0, MU, LAM)
        A = oracle_mod.dpdf(F0, MU, LAM)
        eps = 1e-6
        Pfd = np.zeros((3, 3))
        Afd = np.zeros((9, 9))
        for i in range(3):
            for j in range(3):
                dF = np.zeros((3, 3)); dF[i, j] = eps
                Pfd[i, j] = (oracle_mod.psi(F0 + dF, MU, LAM) - oracle_mod.psi(F0 - dF, MU, LAM)) / (2 * eps)
                dP = (oracle_mod.pk1(F0 + dF, MU, LAM) - oracle_mod.pk1(F0 - dF, MU, LAM)) / (2 * eps)
                Afd[:, 3 * j + i] = dP.T.ravel()  # column-major vec of dP
        assert np.abs(Pfd - P).max() <= 1e-8 * np.abs(P).max()
        assert np.abs(Afd - A).max() <= 1e-8 * np.abs(A).max()
        assert np.allclose(A, A.T, rtol=1e-14, atol=1e-6)


def unit_tet(h=0.1):
    return np.array([[0, 0, 0], [h, 0, 0], [0, h, 0], [0, 0, h]], dtype=float)


def test_element_rest_and_rigid_motion(oracle_mod):
    rng = np.random.default_rng(2)
    Xe = unit_tet() + 0.01 * rng.normal(size=(4, 3))
    Dminv, V = oracle_mod.rest(Xe)
    assert V > 0
    R = rot(rng)
    xe = Xe @ R.T + rng.normal(size=3)
    assert abs(oracle_mod.elem_energy(Xe, xe, MU, LAM)) < 1e-9 * MU * V
    assert np.abs(oracle_mod.elem_grad(Xe, xe, MU, LAM)).max() < 1e-9 * MU * 0.01


def test_element_gradient_hessian_fd_and_nullspace(oracle_mod):
    rng = np.random.default_rng(3)
    Xe = unit_tet()
    xe = Xe + 0.03 * rng.normal(size=(4, 3))
    g = oracle_mod.elem_grad(Xe, xe, MU, LAM)
    H = oracle_mod.elem_hess(Xe, xe, MU, LAM)
    eps = 1e-7
    gfd = np.zeros(12)
    Hfd = np.zeros((12, 12))
    for k in range(12):
        d = np.zeros(12); d[k] = eps
        xp, xm = (xe.ravel() + d).reshape(4, 3), (xe.ravel() - d).reshape(4, 3)
        gfd[k] = (oracle_mod.elem_energy(Xe, xp, MU, LAM) - oracle_mod.elem_energy(Xe, xm, MU, LAM)) / (2 * eps)
        Hfd[:, k] = (oracle_mod.elem_grad(Xe, xp, MU, LAM) - oracle_mod.elem_grad(Xe, xm, MU, LAM)) / (2 * eps)
    assert np.abs(gfd - g).max() <= 1e-7 * np.abs(g).max()
    assert np.abs(Hfd - H).max() <= 1e-7 * np.abs(H).max()
    # translation invariance: gradient rows sum to zero, H (1 (x) t) = 0
    assert np.abs(g.reshape(4, 3).sum(0)).max() <= 1e-12 * np.abs(g).max()
    for t in np.eye(3):
        assert np.abs(H @ np.tile(t, 4)).max() <= 1e-10 * np.abs(H).max()


def test_jacobi_eigen_matches_library(oracle_mod):
    rng = np.random.default_rng(4)
    for n in [1, 5, 16]:
        A = rng.normal(size=(n, n)); A = A + A.T
        w, V = oracle_mod.sym_eig(A)
        wl = np.linalg.eigvalsh(A)
        assert np.allclose(np.sort(w), wl, rtol=1e-12, atol=1e-12)
        assert np.allclose(V @ np.diag(w) @ V.T, A, atol=1e-11)
