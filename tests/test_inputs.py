"""Pins of the synthetic mesh generator and of the oracle's rest-shape data:
counts, volumes, orientation, conformity and mass against closed forms."""
import json
import os
from collections import Counter

import numpy as np
import pytest

from paper_2409_03807_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_mesh_counts_volume_conformity(name, oracle_mod):
    g = GOLD["meshes"][name]
    X, tets = I.cube_grid(g["nx"], g["ny"], g["nz"], g["h"])
    assert X.shape == (g["nv"], 3) and tets.shape == (g["ne"], 4)
    vols = np.array([oracle_mod.rest(X[t])[1] for t in tets])
    h3 = g["h"] ** 3
    assert np.all(vols > 0), "every tet positively oriented"
    ok = np.isclose(vols, h3 / 6, rtol=1e-12) | np.isclose(vols, h3 / 3, rtol=1e-12)
    assert ok.all()
    assert np.isclose(vols.sum(), g["volume"], rtol=1e-12)
    faces = Counter()
    for t in tets:
        for skip in range(4):
            faces[tuple(sorted(int(v) for i, v in enumerate(t) if i != skip))] += 1
    assert max(faces.values()) <= 2, "no face shared by more than two tets"
    assert sum(1 for c in faces.values() if c == 1) == g["boundary_tris"]


def test_total_mass_c1(oracle_mod):
    p = I.config("c1")
    m = oracle_mod.Oracle(p).lumped_mass()
    assert np.isclose(m.sum(), GOLD["meshes"]["c1"]["mass"], rtol=1e-12)
    assert np.all(m > 0)


def test_faces_and_cubature():
    p = I.config("c2")
    assert len(p.target_vtx) == 81 and p.pinned.sum() == 81
    assert np.all(p.X[p.target_vtx, 0] == pytest.approx(1.0))
    assert len(np.unique(p.cub_elem)) == 256
    assert p.cub_w.min() >= 20 and p.cub_w.max() <= 80
    p1 = I.config("c1")
    assert len(p1.cub_elem) == 200 and np.all(p1.cub_w == 1.0)


def test_twist_targets_are_rotations():
    p = I.config("c2")
    t = I.twist_targets(p.X, p.target_vtx, np.array([0.0, 90.0, 180.0]))
    P = p.X[p.target_vtx]
    assert np.allclose(t[0], P)
    c = P.mean(0)
    # distances to the centroid are preserved and 180 deg mirrors y,z
    assert np.allclose(np.linalg.norm(t[1] - c, axis=1), np.linalg.norm(P - c, axis=1))
    assert np.allclose(t[2][:, 1:] - c[1:], -(P[:, 1:] - c[1:]))


def test_c5_contact_set_is_the_free_surface():
    p = I.config("c5")
    X = p.X
    lo, hi = X.min(0), X.max(0)
    on_surface = np.any(np.isclose(X, lo) | np.isclose(X, hi), axis=1)
    cv = p.contact_vtx
    # every contact vertex is a free surface vertex, and every free surface vertex is one
    assert on_surface[cv].all() and not p.pinned[cv].any()
    assert len(cv) == int((on_surface & ~p.pinned.astype(bool)).sum())
    # 50 x 10 x 10 cubes: 51 * 11 * 11 vertices, (49 * 9 * 9) interior, 11 * 11 on the pinned face
    assert len(cv) == 51 * 11 * 11 - 49 * 9 * 9 - 11 * 11


def test_end_pose_targets_are_rigid_motions():
    p = I.config("c5")
    q = I.end_pose_problem(p)
    assert len(q.target_vtx) == 121 and len(q.contact_vtx) == 0 and q.dt == 0.0
    t = I.end_pose_targets(p, q.target_vtx, 6, bend_deg=45.0, twist_deg=60.0)
    P = p.X[q.target_vtx]
    D0 = np.linalg.norm(P[:, None] - P[None], axis=-1)
    c0 = p.X[p.pinned.astype(bool)].mean(0)
    for b in range(6):
        # pairwise distances of the face and its centroid's distance to the pinned face's are kept
        assert np.allclose(np.linalg.norm(t[b][:, None] - t[b][None], axis=-1), D0)
        assert np.isclose(np.linalg.norm(t[b].mean(0) - c0), np.linalg.norm(P.mean(0) - c0))
        # the face's area element is kept (no shear or scaling of the face)
        e1, e2 = P[1] - P[0], P[11] - P[0]
        f1, f2 = t[b][1] - t[b][0], t[b][11] - t[b][0]
        assert np.isclose(np.linalg.norm(np.cross(f1, f2)), np.linalg.norm(np.cross(e1, e2)))
    # nonzero angles move the face
    assert np.abs(t - P[None]).max() > 0.1
    # zero angles leave the face where it is
    t0 = I.end_pose_targets(p, q.target_vtx, 1, bend_deg=0.0, twist_deg=0.0)
    assert np.allclose(t0[0], P)
