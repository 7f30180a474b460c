"""Seeded synthetic inputs for the spectral-element Poisson solver.

This module only draws inputs: vertex coordinates and hexahedron connectivity
of perturbed cube meshes, element permutations, local vertex rotations and
random right-hand sides.  It contains none of the discretisation's arithmetic
(no GLL points, no numbering, no geometry), so both the CPU oracle and the
GPU library can take their inputs from it without sharing any of the method.

Conventions (shared by every consumer):

* vertex ids are lexicographic with x fastest: ``v = a + (kx+1) b + (kx+1)(ky+1) c``;
* a hexahedron lists its 8 vertices in tensor order: local corner ``(a, b, c)``
  with ``a, b, c`` in {0, 1} sits at position ``a + 2 b + 4 c``;
* element ids are lexicographic (x fastest) before an optional permutation.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in this order:
(1) perturbation of the interior vertices, ascending vertex id, x then y then z,
each uniform in ``(-p h_d, +p h_d)``; (2) the element permutation; (3) the
right-hand side.  The paper's own meshes exist only as figures, so perturbed
cubes stand in for them (Section 6.1 uses 8^3..128^3 refinements of a cube).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1506


@dataclass
class HexMesh:
    """Unstructured all-hex mesh: coordinates plus tensor-ordered connectivity."""

    vtx: np.ndarray  # [V, 3] float64
    hex: np.ndarray  # [E, 8] int64, tensor vertex order
    shape: tuple = ()  # (kx, ky, kz) of the generating lattice, for bookkeeping
    lengths: tuple = ()  # domain extents
    perm: np.ndarray | None = None  # element permutation applied (new -> old)
    meta: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.hex.shape[0])

    @property
    def n_vtx(self) -> int:
        return int(self.vtx.shape[0])


def cube_mesh(k, lengths=(1.0, 1.0, 1.0), perturb=0.0, seed=BASE_SEED,
              permute=False, rng=None) -> HexMesh:
    """Box ``[0,Lx]x[0,Ly]x[0,Lz]`` split into ``kx*ky*kz`` hexahedra.

    ``k`` is an int or a 3-tuple.  Interior vertices are moved by independent
    uniform draws in ``(-perturb*h_d, +perturb*h_d)`` per coordinate; boundary
    vertices stay on the box so the domain and its Dirichlet faces are exact.
    With ``permute`` the element ids are shuffled (unstructured indexing).
    """
    if np.isscalar(k):
        k = (int(k),) * 3
    kx, ky, kz = (int(v) for v in k)
    Lx, Ly, Lz = (float(v) for v in lengths)
    if rng is None:
        rng = np.random.default_rng(seed)
    nx, ny, nz = kx + 1, ky + 1, kz + 1
    a = np.arange(nx)
    b = np.arange(ny)
    c = np.arange(nz)
    C, B, A = np.meshgrid(c, b, a, indexing="ij")  # x fastest
    A = A.ravel()
    B = B.ravel()
    C = C.ravel()
    h = np.array([Lx / kx, Ly / ky, Lz / kz])
    vtx = np.stack([A * h[0], B * h[1], C * h[2]], axis=1).astype(np.float64)
    interior = (A > 0) & (A < kx) & (B > 0) & (B < ky) & (C > 0) & (C < kz)
    n_int = int(interior.sum())
    if perturb != 0.0 and n_int > 0:
        d = rng.uniform(-1.0, 1.0, size=(n_int, 3)) * (perturb * h)[None, :]
        vtx[interior] += d
    # connectivity, element ids lexicographic with x fastest
    ez, ey, ex = np.meshgrid(np.arange(kz), np.arange(ky), np.arange(kx), indexing="ij")
    ex = ex.ravel()
    ey = ey.ravel()
    ez = ez.ravel()
    hexes = np.empty((kx * ky * kz, 8), dtype=np.int64)
    for cc, bb, aa in itertools.product((0, 1), (0, 1), (0, 1)):
        hexes[:, aa + 2 * bb + 4 * cc] = (ex + aa) + nx * (ey + bb) + nx * ny * (ez + cc)
    perm = None
    if permute:
        perm = rng.permutation(hexes.shape[0])
        hexes = hexes[perm]
    return HexMesh(vtx=vtx, hex=hexes, shape=(kx, ky, kz), lengths=(Lx, Ly, Lz), perm=perm,
                   meta={"perturb": perturb, "seed": seed})


# --- the 24 proper rotations of the reference cube, as corner permutations ---

def _cube_rotations():
    """All 24 orientation-preserving symmetries of the cube as maps on corner
    positions ``a + 2b + 4c``; each entry ``r`` relabels a hex by
    ``new[pos] = old[r[pos]]``."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), dtype=int)
            for r, (p, s) in enumerate(zip(perm, signs)):
                M[r, p] = s
            if round(np.linalg.det(M)) == 1:
                mats.append(M)
    rots = []
    for M in mats:
        r = np.empty(8, dtype=np.int64)
        for cc, bb, aa in itertools.product((0, 1), (0, 1), (0, 1)):
            x = np.array([2 * aa - 1, 2 * bb - 1, 2 * cc - 1])
            y = M @ x
            a2, b2, c2 = ((y + 1) // 2).tolist()
            r[aa + 2 * bb + 4 * cc] = a2 + 2 * b2 + 4 * c2
        rots.append(r)
    return np.array(rots)


CUBE_ROTATIONS = _cube_rotations()


def rotate_elements(mesh: HexMesh, seed=BASE_SEED + 7) -> tuple[HexMesh, np.ndarray]:
    """Give every hexahedron one of the 24 local orientations, drawn at random.

    Returns the relabelled mesh and the rotation index per element.  The
    geometry and topology are unchanged; only each element's local frame moves.
    """
    rng = np.random.default_rng(seed)
    rot = rng.integers(0, 24, size=mesh.n_elem)
    R = CUBE_ROTATIONS[rot]  # [E, 8]
    hexes = np.take_along_axis(mesh.hex, R, axis=1)
    return HexMesh(vtx=mesh.vtx, hex=hexes, shape=mesh.shape, lengths=mesh.lengths,
                   perm=mesh.perm, meta=dict(mesh.meta, rotated=True)), rot


def permute_elements(mesh: HexMesh, seed=BASE_SEED + 11) -> tuple[HexMesh, np.ndarray]:
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh.n_elem)
    return HexMesh(vtx=mesh.vtx, hex=mesh.hex[perm], shape=mesh.shape, lengths=mesh.lengths,
                   perm=perm, meta=dict(mesh.meta, permuted=True)), perm


def star_mesh(n_sides=5, layers=3, height=1.0, perturb=0.0, seed=BASE_SEED) -> HexMesh:
    """Extruded polygon whose edges have valence other than 4.

    In the plane: a centre C, spoke points S_i (radius 1, angle 2 pi i/n), mid
    points M_i (radius 1.25, angle (2i+1) pi/n), and an outer ring T_i, U_i
    (radii 2.2, 2.4 at the spoke / mid angles).  Quads: kites (C, S_i, S_i+1,
    M_i) and two outer quads per sector, (S_i, T_i, M_i, U_i) and (M_i, U_i,
    S_i+1, T_i+1), listed in tensor order with a right-handed frame.  Interior
    vertices: C (valence n in the plane), S_i (4), M_i (3); extruding into
    ``layers`` slabs of ``height`` gives interior mesh edges of valence n, 4
    and 3.  Interior vertices (not on the outer ring, top or bottom) move by
    uniform draws in (-perturb, +perturb) per coordinate.
    """
    n = int(n_sides)
    ang = 2.0 * np.pi * np.arange(n) / n
    mid = ang + np.pi / n
    pts = [(0.0, 0.0)]
    pts += [(np.cos(a), np.sin(a)) for a in ang]                # S_i: 1 + i
    pts += [(1.25 * np.cos(a), 1.25 * np.sin(a)) for a in mid]  # M_i: 1 + n + i
    pts += [(2.2 * np.cos(a), 2.2 * np.sin(a)) for a in ang]    # T_i: 1 + 2n + i
    pts += [(2.4 * np.cos(a), 2.4 * np.sin(a)) for a in mid]    # U_i: 1 + 3n + i
    P2 = np.array(pts)
    S = lambda i: 1 + (i % n)
    M = lambda i: 1 + n + (i % n)
    T = lambda i: 1 + 2 * n + (i % n)
    U = lambda i: 1 + 3 * n + (i % n)
    quads = []  # tensor order (0,0), (1,0), (0,1), (1,1)
    for i in range(n):
        quads.append((0, S(i), S(i + 1), M(i)))
        quads.append((S(i), T(i), M(i), U(i)))
        quads.append((M(i), U(i), S(i + 1), T(i + 1)))
    np2 = P2.shape[0]
    z = np.linspace(0.0, height, layers + 1)
    vtx = np.array([(x, y, zz) for zz in z for (x, y) in P2], dtype=np.float64)
    hexes = []
    for l in range(layers):
        for q in quads:
            hexes.append([l * np2 + v for v in q] + [(l + 1) * np2 + v for v in q])
    hexes = np.array(hexes, dtype=np.int64)
    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        for v in range(vtx.shape[0]):
            l, p = divmod(v, np2)
            if 0 < l < layers and p < 1 + 2 * n:
                vtx[v] += rng.uniform(-perturb, perturb, size=3)
    return HexMesh(vtx=vtx, hex=hexes, shape=(n, layers), lengths=(4.8, 4.8, height),
                   meta=dict(star=n, layers=layers, perturb=perturb))


def random_vector(n, seed=BASE_SEED + 3, low=-1.0, high=1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(low, high, size=n)


# --- named workloads ------------------------------------------------------

def manufactured_u(xyz, lengths=(1.0, 1.0, 1.0)):
    """Exact solution sin(pi x/Lx') sin(pi y/Ly') sin(pi z/Lz') used by the workloads."""
    Lx, Ly, Lz = lengths
    return (np.sin(np.pi * xyz[..., 0] / Lx) * np.sin(np.pi * xyz[..., 1] / Ly)
            * np.sin(np.pi * xyz[..., 2] / Lz))


def manufactured_s(xyz, lengths=(1.0, 1.0, 1.0)):
    """Source s = -Laplace(u) for :func:`manufactured_u` (kappa=1, c=0)."""
    Lx, Ly, Lz = lengths
    lam = np.pi ** 2 * (1.0 / Lx ** 2 + 1.0 / Ly ** 2 + 1.0 / Lz ** 2)
    return lam * manufactured_u(xyz, lengths)


def mixed_bc_u(xyz):
    """Exact solution sin(pi x) sin(pi y) (z + z^2) on the unit cube: zero on every
    face but z = 1, where its normal derivative is 3 sin(pi x) sin(pi y)."""
    return np.sin(np.pi * xyz[..., 0]) * np.sin(np.pi * xyz[..., 1]) * (xyz[..., 2] + xyz[..., 2] ** 2)


def mixed_bc_s(xyz):
    """Source s = -Laplace(u) of :func:`mixed_bc_u` (kappa = 1, c = 0)."""
    sxy = np.sin(np.pi * xyz[..., 0]) * np.sin(np.pi * xyz[..., 1])
    z = xyz[..., 2]
    return sxy * (2.0 * np.pi ** 2 * (z + z ** 2) - 2.0)


def mixed_bc_g(xyz):
    """Neumann data du/dz of :func:`mixed_bc_u` on z = 1."""
    return 3.0 * np.sin(np.pi * xyz[..., 0]) * np.sin(np.pi * xyz[..., 1])


def top_faces(mesh, tol=1e-12):
    """(element, local face) pairs of the faces lying on z = Lz (local face
    2 axis + side over the element's tensor corners)."""
    Lz = mesh.lengths[2]
    Z = mesh.vtx[mesh.hex][..., 2]  # [E, 8], corner a + 2b + 4c
    on_top = np.abs(Z - Lz) <= tol
    out = []
    for lf in range(6):
        d, side = lf // 2, lf % 2
        corners = [q for q in range(8) if ((q >> d) & 1) == side]
        for e in np.nonzero(on_top[:, corners].all(axis=1))[0]:
            out.append((int(e), lf))
    out.sort()
    return np.array(out, dtype=np.int64).reshape(-1, 2)


# Heat-equation workload: the parameters of the aluminium-rod run (kappa in
# m^2/s, time step in s, a volume source Q over rho c_p) with the source taken
# as a Gaussian blob that travels along the rod's long (z) axis.
HEAT = dict(kappa=1e-2, dt=0.04, steps=70, Q=1000.0, rho=7000.0, cp=0.8, sigma=0.2,
            z_start=0.2, z_end=0.6)


def heat_source(xyz, t, lengths, sigma=HEAT["sigma"], amplitude=HEAT["Q"] / (HEAT["rho"] * HEAT["cp"]),
                z_start=HEAT["z_start"], z_end=HEAT["z_end"], t_end=HEAT["dt"] * HEAT["steps"], exp=np.exp):
    """Nodal source q(x, t): a Gaussian of width sigma centred on the rod axis,
    its centre moving at constant speed from z_start Lz (t = 0) to z_end Lz (t = t_end).
    ``exp`` lets array libraries other than numpy evaluate it on their own arrays."""
    Lx, Ly, Lz = lengths
    zc = Lz * (z_start + (z_end - z_start) * t / t_end)
    d2 = ((xyz[..., 0] - Lx / 2) ** 2 + (xyz[..., 1] - Ly / 2) ** 2 + (xyz[..., 2] - zc) ** 2)
    return amplitude * exp(-d2 / (2.0 * sigma ** 2))


WORKLOADS = {
    # 4^3 hexes of the unit cube, interior vertices +-10% h, order 4 (4913 DOFs)
    "cube4_N4": dict(k=4, lengths=(1.0, 1.0, 1.0), perturb=0.10, N=4, permute=False),
    # 56^3 hexes, +-15% h, random element ids, order 7 (60,698,457 DOFs)
    "cube56_N7": dict(k=56, lengths=(1.0, 1.0, 1.0), perturb=0.15, N=7, permute=True),
    # 20^3 hexes stretched 8:1 in z, +-10% h, order 15 (27,270,901 DOFs)
    "box20x8_N15": dict(k=20, lengths=(1.0, 1.0, 8.0), perturb=0.10, N=15, permute=False),
    # heat-equation rod: 10 x 10 x 625 hexes of a 1 x 1 x 62.5 bar (62,500 hexes,
    # near the 62,540 of the paper's rod), +-10% h, random ids, order 7 (22,059,416 DOFs)
    "rod625_N7": dict(k=(10, 10, 625), lengths=(1.0, 1.0, 62.5), perturb=0.10, N=7, permute=True),
}


def workload_mesh(name: str, seed=BASE_SEED) -> tuple[HexMesh, int]:
    w = WORKLOADS[name]
    m = cube_mesh(w["k"], lengths=w["lengths"], perturb=w["perturb"], seed=seed,
                  permute=w["permute"])
    return m, w["N"]


def batch_instances(n=64, seed=BASE_SEED):
    """Batched workload: instance i uses seed+i to draw (N, k), the mesh
    perturbation (+-10% h) and a right-hand side uniform in (-1, 1) over the
    ``(kN+1)^3`` global nodes (masked to the interior by the caller)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        N = int(rng.integers(3, 9))
        k = int(rng.integers(2, 25))
        mesh = cube_mesh(k, perturb=0.10, rng=rng)
        n_global = (k * N + 1) ** 3
        rhs = rng.uniform(-1.0, 1.0, size=n_global)
        out.append(dict(N=N, k=k, mesh=mesh, rhs=rhs, seed=seed + i))
    return out
