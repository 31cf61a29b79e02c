"""Seeded synthetic inputs for the reduced-Newton hot path.

This module only *generates* arrays: a cube-grid tetrahedral beam, the material
constants as given (Young's modulus, Poisson ratio, density, gravity), Glorot
initialised decoder weights, a cubature draw, latent batches and twist / bend
loads.  It holds none of the method's arithmetic (no rest-shape inverse, no
volumes, no masses, no Lame parameters, no energy): both the GPU library and
the CPU oracle derive those from the arrays built here, each on its own.

The paper runs its method on its own meshes (Table 1: Twist Bar, Dinosaur,
Elephant, Bunny); those meshes are not available, so regular beams made of
cubes split into five tetrahedra stand in for them, with the problem sizes
(n, E, r, S) of the same order as the quasi-static Twist Bar of Table 1.

Seeds: decoder 0, cubature 1, latent batches 2, loads 3, train/held-out split
4, snapshot loads 5, encoder 6.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_DECODER = 0
SEED_CUBATURE = 1
SEED_LATENT = 2
SEED_LOADS = 3
SEED_SPLIT = 4
SEED_SNAPSHOTS = 5
SEED_ENCODER = 6


# ----------------------------------------------------------------------------
# mesh
# ----------------------------------------------------------------------------
def vertex_id(i, j, k, ny, nz):
    return (i * (ny + 1) + j) * (nz + 1) + k


def cube_grid(nx: int, ny: int, nz: int, h: float):
    """Regular grid of nx*ny*nz cubes of edge h, each split into 5 tets.

    Vertex (i,j,k) has id (i*(ny+1)+j)*(nz+1)+k and rest position (ih,jh,kh).
    The split alternates with the parity of i+j+k so that neighbouring cubes
    share face diagonals (a conforming mesh): for even parity the central tet
    uses the four odd-parity corners and each even-parity corner forms a corner
    tet with its three edge neighbours; odd parity swaps the roles.  Each tet
    is listed with positive orientation (the first vertex's three edges form a
    right-handed frame).

    Returns X (nv,3) float64 and tets (ne,4) int32.
    """
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    X = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)
    tets = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                c = {(a, b, d): vertex_id(i + a, j + b, k + d, ny, nz)
                     for a in (0, 1) for b in (0, 1) for d in (0, 1)}
                even = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
                odd = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
                centre, corners = (odd, even) if (i + j + k) % 2 == 0 else (even, odd)
                cube_tets = [centre]
                for v in corners:
                    nb = [tuple(v[t] ^ (1 if t == s else 0) for t in range(3)) for s in range(3)]
                    cube_tets.append([v] + nb)
                for t in cube_tets:
                    ids = [c[v] for v in t]
                    # orientation by the sign of the corner-offset triple product
                    # (pure connectivity bookkeeping on integer offsets)
                    o = [np.array(v) for v in t]
                    e1, e2, e3 = o[1] - o[0], o[2] - o[0], o[3] - o[0]
                    if int(np.dot(e1, np.cross(e2, e3))) < 0:
                        ids[1], ids[2] = ids[2], ids[1]
                    tets.append(ids)
    return X, np.asarray(tets, dtype=np.int32)


def face_vertices(X: np.ndarray, axis: int, value: float, tol: float = 1e-9):
    return np.nonzero(np.abs(X[:, axis] - value) < tol)[0].astype(np.int32)


# ----------------------------------------------------------------------------
# decoder weights
# ----------------------------------------------------------------------------
def glorot_decoder(r: int, hidden: list[int], n_out: int, seed: int = SEED_DECODER,
                   bias_scale: float = 0.0):
    """Glorot-uniform MLP weights, U(+-sqrt(6/(fan_in+fan_out))), drawn layer by
    layer from one generator; biases zero unless bias_scale > 0 (then
    U(+-bias_scale), drawn after all weights).  W[l] has shape (out, in)."""
    rng = np.random.default_rng(seed)
    sizes = [r] + list(hidden) + [n_out]
    Ws, bs = [], []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(6.0 / (fin + fout))
        Ws.append(rng.uniform(-lim, lim, size=(fout, fin)))
    for fout in sizes[1:]:
        if bias_scale > 0:
            bs.append(rng.uniform(-bias_scale, bias_scale, size=fout))
        else:
            bs.append(np.zeros(fout))
    return Ws, bs


def identity_decoder(free_dofs: np.ndarray, n_out: int):
    """Linear decoder (no hidden layer) whose output selects the free DOFs:
    u = W z with W[free_dofs[k], k] = 1."""
    r = len(free_dofs)
    W = np.zeros((n_out, r))
    W[free_dofs, np.arange(r)] = 1.0
    return [W], [np.zeros(n_out)]


# ----------------------------------------------------------------------------
# cubature, latent batches, loads
# ----------------------------------------------------------------------------
def draw_cubature(ne: int, n_cub: int, wlo: float, whi: float, seed: int = SEED_CUBATURE):
    """n_cub distinct elements drawn uniformly without replacement (sorted), and
    i.i.d. weights U[wlo, whi].  n_cub >= ne gives every element weight 1."""
    if n_cub >= ne:
        return np.arange(ne, dtype=np.int32), np.ones(ne)
    rng = np.random.default_rng(seed)
    elem = np.sort(rng.choice(ne, size=n_cub, replace=False)).astype(np.int32)
    w = rng.uniform(wlo, whi, size=n_cub)
    return elem, w


def latent_batch(B: int, r: int, sigma: float = 0.5, seed: int = SEED_LATENT):
    return np.random.default_rng(seed).normal(0.0, sigma, size=(B, r))


def twist_targets(X: np.ndarray, verts: np.ndarray, angles_deg: np.ndarray):
    """Targets for the end-face vertices rotated about the beam (x) axis through
    the face centroid by each angle.  Returns (B, len(verts), 3)."""
    P = X[verts]
    c = P.mean(axis=0)
    out = np.empty((len(angles_deg), len(verts), 3))
    for b, a in enumerate(np.deg2rad(np.asarray(angles_deg, dtype=np.float64))):
        ca, sa = math.cos(a), math.sin(a)
        d = P - c
        out[b, :, 0] = P[:, 0]
        out[b, :, 1] = c[1] + ca * d[:, 1] - sa * d[:, 2]
        out[b, :, 2] = c[2] + sa * d[:, 1] + ca * d[:, 2]
    return out


def twist_sweep(B: int, sweep=(0.0, 45.0, 90.0, 135.0, 180.0)):
    return np.asarray([sweep[b % len(sweep)] for b in range(B)], dtype=np.float64)


def bend_forces(B: int, n_verts: int, fmax: float = 2000.0, seed: int = SEED_LOADS):
    """Per-vertex force on each load vertex: a total |F| ~ U[0, fmax] N in a
    random direction of the y-z plane, spread equally over n_verts."""
    rng = np.random.default_rng(seed)
    mag = rng.uniform(0.0, fmax, size=B)
    ang = rng.uniform(0.0, 2 * math.pi, size=B)
    f = np.zeros((B, 3))
    f[:, 1] = mag * np.cos(ang) / n_verts
    f[:, 2] = mag * np.sin(ang) / n_verts
    return f


# ----------------------------------------------------------------------------
# workload presets
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    """Every array one reduced problem needs, in plain float64/int32 form."""
    name: str
    X: np.ndarray            # (nv,3)
    tets: np.ndarray         # (ne,4) int32
    pinned: np.ndarray       # (nv,) uint8, 1 = Dirichlet-fixed at rest
    young: float
    poisson: float
    density: float
    gravity: np.ndarray      # (3,)
    r: int
    hidden: list
    Ws: list                 # W[l] (out,in)
    bs: list
    cub_elem: np.ndarray     # (S,) int32
    cub_w: np.ndarray        # (S,)
    target_vtx: np.ndarray   # (nt,) int32  penalty-constrained vertices
    k_c: float
    force_vtx: np.ndarray    # (nf,) int32  vertices that receive the bend force
    meta: dict = field(default_factory=dict)
    # implicit Euler (dt > 0) and ground contact on contact_vtx (plane y = ground_y)
    dt: float = 0.0
    contact_vtx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    k_ground: float = 0.0
    ground_y: float = 0.0

    @property
    def nv(self):
        return self.X.shape[0]

    @property
    def ne(self):
        return self.tets.shape[0]

    @property
    def n(self):
        return 3 * self.nv


def make_problem(name: str, nx, ny, nz, r, hidden, n_cub, wlo=20.0, whi=80.0,
                 k_c=1e6, gravity=True, twist=True, bend=False,
                 length=1.0, bias_scale=0.0, decoder_seed=SEED_DECODER):
    h = length / nx
    X, tets = cube_grid(nx, ny, nz, h)
    nv = X.shape[0]
    pinned = np.zeros(nv, dtype=np.uint8)
    pinned[face_vertices(X, 0, 0.0)] = 1
    end = face_vertices(X, 0, nx * h)
    Ws, bs = glorot_decoder(r, hidden, 3 * nv, seed=decoder_seed, bias_scale=bias_scale)
    cub_elem, cub_w = draw_cubature(tets.shape[0], n_cub, wlo, whi)
    g = np.array([0.0, -9.81, 0.0]) if gravity else np.zeros(3)
    return Problem(name=name, X=X, tets=tets, pinned=pinned, young=1e5, poisson=0.45,
                   density=1000.0, gravity=g, r=r, hidden=list(hidden), Ws=Ws, bs=bs,
                   cub_elem=cub_elem, cub_w=cub_w,
                   target_vtx=end if twist else np.zeros(0, np.int32), k_c=k_c,
                   force_vtx=end if bend else np.zeros(0, np.int32),
                   meta=dict(nx=nx, ny=ny, nz=nz, h=h))


def config(name: str, **kw) -> Problem:
    """The workloads of the reduced solver.

    c1: 10x2x2 beam (99 vertices, 200 tets, n=297), r=8, 3x64 ELU, all tets as
        cubature with weight 1, gravity, x=0 face fixed; FP64.
    c2: 40x8x8 beam (3321 vertices, 12800 tets, n=9963), r=16, 4x128 ELU, 256
        cubature tets with weights U[20,80], end twist 0-180 deg as penalty
        targets (k_c = 1e6 N/m) on the x=L face; FP32 path, batch 1024.
    c3: c2 with batch 4096 (BF16 decoder variant).
    c4: 16^3 block (4913 vertices, 20480 tets), r=12, 4x256, 512 cubature tets
        with weights U[20,60], end twist and bend loads on the x=L face.
    c5: 50x10x10 beam (6171 vertices, 25000 tets), r=32, 5x256, 1024 cubature tets
        (weights with mean ne / |S|); implicit Euler dt = 1/60, ground plane
        y = -0.25 m with penalty stiffness 1e6 N/m on the free surface vertices
        (2081: the solid's interior reaches the plane only after its surface).
    """
    name = name.lower()
    if name == "c1":
        return make_problem("c1", 10, 2, 2, 8, [64] * 3, 10 ** 9, twist=False, **kw)
    if name in ("c2", "c3"):
        return make_problem(name, 40, 8, 8, 16, [128] * 4, 256, **kw)
    if name == "c4":
        # weights U[20, 60]: mean 40 = ne / |S|, so the cubature sum has the element count's scale
        return make_problem("c4", 16, 16, 16, 12, [256] * 4, 512, wlo=20.0, whi=60.0, bend=True, **kw)
    if name == "c5":
        # implicit-Euler dynamics: x = 0 face pinned, gravity, ground contact on every vertex
        p = make_problem("c5", 50, 10, 10, 32, [256] * 5, 1024, wlo=12.5, whi=36.3, twist=False, **kw)
        p.dt = 1.0 / 60.0
        lo, hi = p.X.min(axis=0), p.X.max(axis=0)
        surf = np.any(np.isclose(p.X, lo) | np.isclose(p.X, hi), axis=1) & ~p.pinned.astype(bool)
        p.contact_vtx = np.nonzero(surf)[0].astype(np.int32)
        p.k_ground = 1e6
        p.ground_y = -0.25
        return p
    if name == "tiny":
        # 2x1x1 beam, r=4, 2x8 hidden, 8 of the 10 tets as cubature, weights U[20,80]
        return make_problem("tiny", 2, 1, 1, 4, [8, 8], 8, **kw)
    raise ValueError(f"unknown config {name}")


def loads_for(p: Problem, B: int, twist_deg=None, seed: int = SEED_LOADS):
    """(targets (B,nt,3) or None, force (B,3) or None) for a batch."""
    targets = None
    force = None
    if len(p.target_vtx):
        ang = twist_sweep(B) if twist_deg is None else np.broadcast_to(
            np.asarray(twist_deg, dtype=np.float64), (B,))
        targets = twist_targets(p.X, p.target_vtx, ang)
    if len(p.force_vtx):
        force = bend_forces(B, len(p.force_vtx), seed=seed)
    return targets, force


def snapshot_loads(p: Problem, N: int, seed: int = SEED_SNAPSHOTS, fmax: float = 2000.0):
    """Load cases of the snapshot set: end twist U[-180, 180] deg (penalty targets
    on the x = L face) and a bend load |F| ~ U[0, fmax] N in a random direction of
    the y-z plane spread over the same face.  Returns (twist (N,), targets
    (N, nt, 3), force per loaded vertex (N, 3))."""
    rng = np.random.default_rng(seed)
    twist = rng.uniform(-180.0, 180.0, size=N)
    mag = rng.uniform(0.0, fmax, size=N)
    ang = rng.uniform(0.0, 2 * math.pi, size=N)
    f = np.zeros((N, 3))
    nf = max(len(p.force_vtx), 1)
    f[:, 1] = mag * np.cos(ang) / nf
    f[:, 2] = mag * np.sin(ang) / nf
    return twist, twist_targets(p.X, p.target_vtx, twist), f


def end_pose_problem(p: Problem) -> Problem:
    """The static snapshot problem of a dynamics workload: the same mesh, material,
    cubature and decoder, with penalty targets (k_c = 1e6 N/m) on the x = L face
    and no inertia or contact (the full-space snapshot solver is quasi-static)."""
    q = Problem(**{**p.__dict__})
    q.target_vtx = face_vertices(p.X, 0, p.X[:, 0].max())
    q.k_c = 1e6
    q.force_vtx = np.zeros(0, np.int32)
    q.contact_vtx = np.zeros(0, np.int32)
    q.dt, q.k_ground = 0.0, 0.0
    return q


def end_pose_targets(p: Problem, verts: np.ndarray, N: int, seed: int = SEED_SNAPSHOTS,
                     bend_deg: float = 60.0, twist_deg: float = 90.0):
    """Targets of the end-face vertices carried rigidly by a rotation about the
    pinned face's centroid: bends about y and z U[-bend_deg, bend_deg], then a
    twist about x U[-twist_deg, twist_deg] through the end face's centroid.
    Returns (N, len(verts), 3)."""
    rng = np.random.default_rng(seed)
    ang = np.deg2rad(rng.uniform(-1.0, 1.0, size=(N, 3)) * np.array([twist_deg, bend_deg, bend_deg]))
    c0 = p.X[p.pinned.astype(bool)].mean(axis=0)
    P = p.X[verts]
    ce = P.mean(axis=0)
    out = np.empty((N, len(verts), 3))
    for b in range(N):
        ax, ay, az = ang[b]
        Rx = np.array([[1, 0, 0], [0, math.cos(ax), -math.sin(ax)], [0, math.sin(ax), math.cos(ax)]])
        Ry = np.array([[math.cos(ay), 0, math.sin(ay)], [0, 1, 0], [-math.sin(ay), 0, math.cos(ay)]])
        Rz = np.array([[math.cos(az), -math.sin(az), 0], [math.sin(az), math.cos(az), 0], [0, 0, 1]])
        R = Rz @ Ry
        tw = ce + (P - ce) @ Rx.T
        out[b] = c0 + (tw - c0) @ R.T
    return out


def heldout_split(N: int, n_test: int, seed: int = SEED_SPLIT):
    """(train indices, held-out indices), a seeded permutation."""
    perm = np.random.default_rng(seed).permutation(N)
    return np.sort(perm[n_test:]), np.sort(perm[:n_test])


def swing_velocities(p: Problem, B: int, seed: int = SEED_LOADS, wmax: float = 6.0):
    """Initial velocities of B simulations: a rigid rotation about the pinned
    face's centre with a seeded rate vector (rad/s, components U[-wmax, wmax]
    about y and z, half that about the beam axis), zero on pinned vertices.
    Returns (B, nv, 3)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(-wmax, wmax, size=(B, 3)) * np.array([0.5, 1.0, 1.0])
    c = p.X[p.pinned.astype(bool)].mean(axis=0)
    d = p.X - c
    v = np.cross(w[:, None, :], d[None, :, :])
    v[:, p.pinned.astype(bool)] = 0.0
    return v

