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
