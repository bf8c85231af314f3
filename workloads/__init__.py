"""Seeded synthetic workloads: meshes, nuclei and random starting blocks.

This module produces *inputs only*.  It holds none of the method's arithmetic
(no assembly, no quadrature, no iteration); both the CPU oracle and the HIP
library consume what it returns.  Every random draw goes through
``numpy.random.default_rng(seed)`` (PCG64), so a seed fully determines a
workload.

Meshes are tensor-product grids split into tetrahedra (Kuhn/Freudenthal split,
six tetrahedra per hexahedral cell).  Graded grids follow the mesh-size law of
Section 4.2 (eq. meshsizefunction), h = min_j(gamma1 Z_j^{-2/5} r_j^{6/5},
gamma2), applied per axis with r_j the distance along that axis, which is a
lower bound on the 3-D distance and therefore refines at least as much as the
law asks.  Nodes on the boundary of the box carry the homogeneous Dirichlet
condition of the H^1_0 space (Section 2.2).

Unstructured graded meshes (the kind the paper builds with a mesh generator
from the same law) apply the law in 3-D distance to an octree, jitter its
vertices and join them by a Delaunay tetrahedralization.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Mesh",
    "Workload",
    "uniform_axis",
    "graded_axis",
    "kuhn_mesh",
    "unstructured_mesh",
    "unstructured_mesh_for_dofs",
    "tet_quality",
    "sample_cluster",
    "random_block",
    "random_block_chunks",
    "make_workload",
    "CONFIGS",
]


@dataclasses.dataclass
class Mesh:
    """Tetrahedral mesh.

    xyz:       float64 [n_nodes, 3] node coordinates (bohr)
    tets:      int32   [n_tets, 4]  node indices of each tetrahedron
    dirichlet: uint8   [n_nodes]    1 on the boundary of the box, else 0
    cells:     (nx, ny, nz) cells per axis of the underlying tensor grid
    """

    xyz: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    cells: tuple

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_dofs(self) -> int:
        return int(self.n_nodes - int(self.dirichlet.sum()))


@dataclasses.dataclass
class Workload:
    """A complete problem instance (inputs only)."""

    name: str
    mesh: Mesh
    Z: np.ndarray          # float64 [M] nuclear charges
    R: np.ndarray          # float64 [M, 3] nuclear positions
    p: int                 # number of orbitals (columns of X)
    beta: float            # penalty parameter of the augmented Lagrangian
    scf: bool              # True: H depends on X (full Kohn-Sham); False: fixed H
    seed: int
    notes: str = ""


# ----------------------------------------------------------------------------
# 1-D grids
# ----------------------------------------------------------------------------

def uniform_axis(lo: float, hi: float, cells: int) -> np.ndarray:
    return np.linspace(lo, hi, cells + 1)


def _merge_anchors(anchors: Sequence[float], zs: Sequence[float], gap: float):
    order = np.argsort(anchors)
    out_a: List[float] = []
    out_z: List[float] = []
    for i in order:
        a, z = float(anchors[i]), float(zs[i])
        if out_a and a - out_a[-1] < gap:
            out_z[-1] = max(out_z[-1], z)
            continue
        out_a.append(a)
        out_z.append(z)
    return np.array(out_a), np.array(out_z)


def graded_axis(lo: float, hi: float, anchors: Sequence[float], zs: Sequence[float],
                gamma1: float, gamma2: float, hmin: float, samples: int = 4096) -> np.ndarray:
    """Node coordinates on [lo, hi] graded by the per-axis mesh-size law.

    Every anchor (a nuclear coordinate on this axis) becomes a node.  Between
    consecutive anchors the cell count is ceil(int dx / h(x)) and nodes are
    placed at equal increments of int dx / h(x).
    """
    a, z = _merge_anchors(anchors, zs, hmin)
    keep = (a > lo + hmin) & (a < hi - hmin)
    a, z = a[keep], z[keep]
    breaks = np.concatenate([[lo], a, [hi]])

    def h_of(x: np.ndarray) -> np.ndarray:
        h = np.full_like(x, gamma2)
        for aj, zj in zip(a, z):
            h = np.minimum(h, gamma1 * zj ** (-0.4) * np.abs(x - aj) ** 1.2)
        return np.clip(h, hmin, gamma2)

    nodes = [lo]
    for s0, s1 in zip(breaks[:-1], breaks[1:]):
        x = np.linspace(s0, s1, samples)
        inv = 1.0 / h_of(x)
        F = np.concatenate([[0.0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(x))])
        ncell = max(1, int(math.ceil(F[-1] - 1e-9)))
        targets = np.linspace(0.0, F[-1], ncell + 1)[1:]
        xs = np.interp(targets, F, x)
        xs[-1] = s1
        nodes.extend(xs.tolist())
    return np.asarray(nodes, dtype=np.float64)


# ----------------------------------------------------------------------------
# Tensor grid -> Kuhn tetrahedra
# ----------------------------------------------------------------------------

# The six tetrahedra of the unit cube that share the diagonal (0,0,0)-(1,1,1):
# one per ordering of the three axes, walking one axis at a time.
_KUHN_PATHS = []
for _perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
    _c = [0, 0, 0]
    _path = [tuple(_c)]
    for _ax in _perm:
        _c[_ax] = 1
        _path.append(tuple(_c))
    _KUHN_PATHS.append(_path)


def _morton_code(I: np.ndarray, J: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Z-order (bit-interleaved) code of each (i, j, k), 21 bits per axis."""
    code = np.zeros(I.shape, dtype=np.uint64)
    for b in range(21):
        for d, A in enumerate((I, J, K)):
            code |= ((A.astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return code


def _morton_rank(I: np.ndarray, J: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Rank of each (i, j, k) along the Z-order (bit-interleaved) curve."""
    order = np.argsort(_morton_code(I, J, K), kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    return rank


def kuhn_mesh(xs: np.ndarray, ys: np.ndarray, zs: np.ndarray, order: str = "morton") -> Mesh:
    """Tensor grid split into 6 tetrahedra per cell.

    order = "morton": nodes are numbered along the Z-order curve of their grid
    indices, so that the neighbours of a node have nearby numbers at every
    scale (the locality a reordered unstructured mesh would have);
    order = "lex": x fastest, then y, then z."""
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    X, Y, Zc = np.meshgrid(xs, ys, zs, indexing="ij")
    # node id = i + (nx+1) * (j + (ny+1) * k)
    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                    Zc.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    n_cells = ci.size
    tets = np.empty((n_cells, 6, 4), dtype=np.int64)
    for t, path in enumerate(_KUHN_PATHS):
        for v, (dx, dy, dz) in enumerate(path):
            tets[:, t, v] = nid(ci + dx, cj + dy, ck + dz)
    tets = tets.reshape(-1, 4).astype(np.int32)

    ii = np.arange(nx + 1)
    jj = np.arange(ny + 1)
    kk = np.arange(nz + 1)
    I, J, K = np.meshgrid(ii, jj, kk, indexing="ij")
    I = I.transpose(2, 1, 0).ravel()
    J = J.transpose(2, 1, 0).ravel()
    K = K.transpose(2, 1, 0).ravel()
    bnd = (I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)
    if order == "morton":
        rank = _morton_rank(I, J, K)              # new id of lexicographic node
        xyz_new = np.empty_like(xyz)
        xyz_new[rank] = xyz
        bnd_new = np.empty_like(bnd)
        bnd_new[rank] = bnd
        tets = rank[tets].astype(np.int32)
        # tetrahedra follow the order of their first vertex
        tets = tets[np.argsort(tets.min(axis=1), kind="stable")]
        xyz, bnd = xyz_new, bnd_new
    elif order != "lex":
        raise ValueError(order)
    return Mesh(xyz=xyz, tets=tets, dirichlet=bnd.astype(np.uint8), cells=(nx, ny, nz))


def graded_mesh(half: float, Z: np.ndarray, R: np.ndarray, gamma1: float, gamma2: float,
                hmin: float) -> Mesh:
    axes = [graded_axis(-half, half, R[:, d], Z, gamma1, gamma2, hmin) for d in range(3)]
    return kuhn_mesh(*axes)


def graded_mesh_for_dofs(half: float, Z: np.ndarray, R: np.ndarray, target_dofs: int,
                         gamma2: float, hmin: float, iters: int = 40) -> tuple:
    """Bisection on gamma1 so that the interior DOF count is close to target."""

    def dofs(g1):
        ax = [graded_axis(-half, half, R[:, d], Z, g1, gamma2, hmin) for d in range(3)]
        return int(np.prod([len(a) - 2 for a in ax]))

    lo, hi = 1e-3, 50.0          # dofs(lo) large, dofs(hi) small
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if dofs(mid) > target_dofs:
            lo = mid
        else:
            hi = mid
    g1 = lo if abs(dofs(lo) - target_dofs) <= abs(dofs(hi) - target_dofs) else hi
    return graded_mesh(half, Z, R, g1, gamma2, hmin), g1


# ----------------------------------------------------------------------------
# Unstructured graded meshes
# ----------------------------------------------------------------------------

def _mesh_size(C: np.ndarray, half_edge: float, Z, R, gamma1: float, gamma2: float,
               hmin: float) -> np.ndarray:
    """The mesh-size law h = min_j(gamma1 Z_j^{-2/5} r_j^{6/5}, gamma2), clipped
    below at hmin, at its smallest over each axis-aligned cube (centre C, half
    edge half_edge): r_j is the distance from nucleus j to the cube."""
    h = np.full(len(C), float(gamma2))
    for Rj, Zj in zip(R, Z):
        d = np.maximum(np.abs(C - Rj) - half_edge, 0.0)
        h = np.minimum(h, gamma1 * float(Zj) ** (-0.4) * np.linalg.norm(d, axis=1) ** 1.2)
    return np.clip(h, hmin, gamma2)


def octree_lattice(half: float, Z, R, gamma1: float, gamma2: float, hmin: float):
    """Vertices of an octree over [-half, half]^3 whose cubes are refined until
    their edge is at most the mesh-size law's h over the cube (or halving would
    go below hmin).  Returns (P, smin, unit, nmax): integer lattice
    coordinates [N, 3] of the distinct cube corners, the edge (in lattice units)
    of the smallest cube at each corner, the lattice step, and the lattice
    size per axis."""
    n0 = max(1, int(math.ceil(2.0 * half / gamma2)))
    s = 2.0 * half / n0
    g = (np.arange(n0) + 0.5) * s - half
    C = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    octants = np.array([[dx, dy, dz] for dx in (-1, 1) for dy in (-1, 1) for dz in (-1, 1)], dtype=np.float64)
    leaves = []
    level = 0
    while len(C):
        split = (s > _mesh_size(C, 0.5 * s, Z, R, gamma1, gamma2, hmin)) & (0.5 * s >= hmin)
        leaves.append((C[~split], level))
        C = (C[split][:, None, :] + 0.25 * s * octants[None]).reshape(-1, 3)
        s *= 0.5
        level += 1
    finest = level - 1
    unit = 2.0 * half / (n0 * 2 ** finest)
    nmax = n0 * 2 ** finest
    corners = np.array([[dx, dy, dz] for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)], dtype=np.int64)
    pts, sizes = [], []
    for Cl, lv in leaves:
        if len(Cl):
            m = 2 ** (finest - lv)
            lo = np.rint((Cl + half) / unit - 0.5 * m).astype(np.int64)
            pts.append((lo[:, None, :] + corners[None] * m).reshape(-1, 3))
            sizes.append(np.full(8 * len(Cl), m, dtype=np.int64))
    P = np.concatenate(pts)
    S = np.concatenate(sizes)
    key = (P[:, 0] * (nmax + 1) + P[:, 1]) * (nmax + 1) + P[:, 2]
    uk, inv = np.unique(key, return_inverse=True)
    smin = np.full(len(uk), np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(smin, inv, S)
    Pu = np.empty((len(uk), 3), dtype=np.int64)
    Pu[inv] = P
    return Pu, smin, unit, nmax


def tet_quality(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """6 sqrt(2) |K| / (longest edge)^3: 1 for the regular tetrahedron, -> 0
    for a flat one."""
    v = xyz[tets]
    vol = np.abs(np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))) / 6.0
    e = np.stack([np.linalg.norm(v[:, a] - v[:, b], axis=1)
                  for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))], axis=1)
    return 6.0 * math.sqrt(2.0) * vol / e.max(axis=1) ** 3


def unstructured_mesh(half: float, Z, R, gamma1: float, gamma2: float, hmin: float, seed: int = 0,
                      jitter: float = 0.3, qmin: float = 0.02, rounds: int = 12, progress=None) -> Mesh:
    """Unstructured graded tetrahedral mesh of [-half, half]^3 following the
    mesh-size law in 3-D distance.

    The octree's cube corners (octree_lattice) are moved by a seeded uniform
    offset of up to jitter x the smallest adjacent cube edge per coordinate
    (points on the box faces move only within their face), then joined by
    the Delaunay tetrahedralization (scipy.spatial.Delaunay, Qhull).  Slivers
    (quality below qmin) are removed by drawing new offsets for their
    interior vertices and triangulating again, for at most `rounds` rounds.
    Nodes are numbered along the Z-order curve of their lattice coordinates
    (neighbours get nearby numbers), tetrahedra are positively oriented and
    ordered by their lowest node.  Nodes on the box faces carry the
    homogeneous Dirichlet condition.  progress(str), if given, is called
    after each triangulation."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    P, smin, unit, nmax = octree_lattice(half, Z, R, gamma1, gamma2, hmin)
    order = np.argsort(_morton_code(P[:, 0], P[:, 1], P[:, 2]), kind="stable")
    P, smin = P[order], smin[order]
    fixed = (P == 0) | (P == nmax)
    onb = fixed.any(axis=1)
    amp = jitter * smin * unit

    def draw(idx):
        J = rng.uniform(-1.0, 1.0, (len(idx), 3)) * amp[idx, None]
        J[fixed[idx]] = 0.0
        return J

    off = draw(np.arange(len(P)))
    for _ in range(rounds + 1):
        xyz = P * unit - half + off
        T = Delaunay(xyz).simplices.astype(np.int64)
        q = tet_quality(xyz, T)
        bad = np.unique(T[q < qmin].ravel())
        bad = bad[~onb[bad]]
        if progress:
            progress(f"Delaunay: {len(P)} points, {len(T)} tetrahedra, quality min {q.min():.3g}, "
                     f"{len(bad)} vertices of slivers")
        if not len(bad):
            break
        off[bad] = draw(bad)
    if q.min() <= 0.0:
        raise RuntimeError("degenerate tetrahedron in the Delaunay mesh")
    v = xyz[T]
    det = np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    neg = det < 0
    T[neg] = T[neg][:, [0, 2, 1, 3]]
    T = T[np.argsort(T.min(axis=1), kind="stable")]
    return Mesh(xyz=xyz, tets=T.astype(np.int32), dirichlet=onb.astype(np.uint8), cells=())


def unstructured_mesh_for_dofs(half: float, Z, R, target_dofs: int, gamma2: float, hmin: float,
                               seed: int = 0, iters: int = 30, progress=None, **mesh_kw) -> tuple:
    """Bisection on gamma1 so that the interior node count of the octree
    lattice is close to target_dofs, then unstructured_mesh (mesh_kw: its
    jitter, qmin, rounds)."""

    def dofs(g1):
        P, _, _, nmax = octree_lattice(half, Z, R, g1, gamma2, hmin)
        return int(np.sum(~((P == 0) | (P == nmax)).any(axis=1)))

    lo, hi = 1e-3, 50.0
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if dofs(mid) > target_dofs:
            lo = mid
        else:
            hi = mid
    g1 = lo if abs(dofs(lo) - target_dofs) <= abs(dofs(hi) - target_dofs) else hi
    if progress:
        progress(f"mesh-size law: gamma1 = {g1:.4g}")
    return unstructured_mesh(half, Z, R, g1, gamma2, hmin, seed=seed, progress=progress, **mesh_kw), g1


# ----------------------------------------------------------------------------
# Nuclei and random blocks
# ----------------------------------------------------------------------------

def sample_cluster(seed: int, M: int, zset: Sequence[int], half_box: float,
                   min_sep: float, max_tries: int = 1_000_000):
    """M nuclei with charges drawn uniformly from zset, positions uniform in
    [-half_box, half_box]^3 by rejection so that every pair is >= min_sep apart."""
    rng = np.random.default_rng(seed)
    Z = rng.choice(np.asarray(zset, dtype=np.float64), size=M)
    R = np.empty((M, 3))
    k = 0
    tries = 0
    while k < M:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place nuclei with the requested separation")
        c = rng.uniform(-half_box, half_box, size=3)
        if k == 0 or np.min(np.linalg.norm(R[:k] - c, axis=1)) >= min_sep:
            R[k] = c
            k += 1
    return Z, R


def random_block(seed: int, n: int, p: int) -> np.ndarray:
    """i.i.d. N(0,1) block, row-major n x p (a node's p values contiguous)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, p))


def device_random_block(seed: int, n: int, p: int, device: str = "cuda"):
    """i.i.d. N(0,1) block (n x p, row-major, float64) drawn on the device by
    torch's seeded generator, for blocks too large to draw and upload from the
    host; the rows an oracle check needs are copied back from it."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((n, p), dtype=torch.float64, device=device, generator=g)


def random_block_chunks(seed: int, n: int, p: int, chunk_rows: int = 1 << 18):
    """The rows of random_block(seed, n, p) in consecutive chunks (r0, r1, rows),
    for blocks too large to hold at once; the same numbers as one call."""
    rng = np.random.default_rng(seed)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        yield r0, r1, rng.standard_normal((r1 - r0, p))


# ----------------------------------------------------------------------------
# The named workloads
# ----------------------------------------------------------------------------

def _c1(seed: int = 0, cells: int = 16) -> Workload:
    ax = uniform_axis(-10.0, 10.0, cells)
    mesh = kuhn_mesh(ax, ax, ax)
    h = 20.0 / cells
    Z = np.array([2.0])
    R = np.array([[0.5 * h, 0.5 * h, 0.5 * h]])     # centre of the cell [0,h]^3
    return Workload("c1", mesh, Z, R, p=4, beta=10.0, scf=False, seed=seed,
                    notes=f"uniform {cells}^3 cells on [-10,10]^3, Z=2 at a cell centre")


def _c2(seed: int = 0, target_dofs: int = 200_000) -> Workload:
    Z, R = sample_cluster(seed, 4, (1, 6, 8), 3.0, 2.0)
    mesh, g1 = graded_mesh_for_dofs(10.0, Z, R, target_dofs, gamma2=1.5, hmin=0.05)
    p = int(math.ceil(Z.sum() / 2.0))
    return Workload("c2", mesh, Z, R, p=p, beta=1.0, scf=True, seed=seed,
                    notes=f"4 nuclei, graded, gamma1={g1:.4g}")


def _cluster_box(M: int) -> float:
    # keep the nuclear number density of 4 nuclei in [-3,3]^3
    return 3.0 * (M / 4.0) ** (1.0 / 3.0)


def _c3(seed: int = 0, target_dofs: int = 2_000_000, p: int = 128, M: int = 24) -> Workload:
    a = _cluster_box(M)
    Z, R = sample_cluster(seed, M, (1, 6, 7, 8), a, 2.0)
    mesh, g1 = graded_mesh_for_dofs(a + 7.0, Z, R, target_dofs, gamma2=1.5, hmin=0.05)
    return Workload("c3", mesh, Z, R, p=p, beta=1.0, scf=False, seed=seed,
                    notes=f"{M} nuclei in [-{a:.3g},{a:.3g}]^3, graded, gamma1={g1:.4g}")


def _c4(seed: int = 0, target_dofs: int = 8_000_000, p: int = 512) -> Workload:
    w = _c3(seed, target_dofs=target_dofs, p=p, M=96)
    w.name = "c4"
    return w


def _u2(seed: int = 0, target_dofs: int = 200_000, progress=None) -> Workload:
    Z, R = sample_cluster(seed, 4, (1, 6, 8), 3.0, 2.0)
    mesh, g1 = unstructured_mesh_for_dofs(10.0, Z, R, target_dofs, gamma2=1.5, hmin=0.05, seed=seed,
                                          progress=progress)
    p = int(math.ceil(Z.sum() / 2.0))
    return Workload("u2", mesh, Z, R, p=p, beta=1.0, scf=True, seed=seed,
                    notes=f"4 nuclei, unstructured graded (Delaunay), gamma1={g1:.4g}")


def _u3(seed: int = 0, target_dofs: int = 500_000, p: int = 128, M: int = 24, progress=None) -> Workload:
    a = _cluster_box(M)
    Z, R = sample_cluster(seed, M, (1, 6, 7, 8), a, 2.0)
    mesh, g1 = unstructured_mesh_for_dofs(a + 7.0, Z, R, target_dofs, gamma2=1.5, hmin=0.05, seed=seed,
                                          progress=progress)
    return Workload("u3", mesh, Z, R, p=p, beta=1.0, scf=False, seed=seed,
                    notes=f"{M} nuclei in [-{a:.3g},{a:.3g}]^3, unstructured graded (Delaunay), gamma1={g1:.4g}")


def make_workload(name: str, seed: int = 0, **kw) -> Workload:
    name = name.lower()
    if name == "u2":
        return _u2(seed, **kw)
    if name == "u3":
        return _u3(seed, **kw)
    if name == "c1":
        return _c1(seed, **kw)
    if name == "c2":
        return _c2(seed, **kw)
    if name in ("c3", "c5"):
        w = _c3(seed, **kw)
        w.name = name
        return w
    if name == "c4":
        return _c4(seed, **kw)
    raise ValueError(f"unknown workload {name!r}")


CONFIGS = {
    "c1": "uniform Kuhn grid 16^3 on [-10,10]^3, Z=2 at a cell centre, p=4, beta=10, fixed H",
    "c2": "4 nuclei Z in {1,6,8} in [-3,3]^3 (sep>=2), graded grid n~2e5, p=ceil(sum Z/2), full SCF LDA",
    "c3": "24 nuclei Z in {1,6,7,8}, graded grid n~2e6, p=128, fixed H (precision form)",
    "c4": "96 nuclei, graded grid n~8e6, p=512, fixed H (precision form at scale)",
    "c5": "c3-type held-out clusters (seeds 2000..2019), learned-preconditioner evaluation",
    "u2": "c2's 4-nucleus clusters on an unstructured graded Delaunay mesh, n~2e5, full SCF LDA",
    "u3": "c3's 24-nucleus clusters on an unstructured graded Delaunay mesh, n~5e5, p=128, fixed H",
}
