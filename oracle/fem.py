"""Oracle: P1 finite-element discretization (Section 2.2).

TEST INFRASTRUCTURE ONLY -- imported by tests/, the smoke check and the CPU
baseline of the benchmark; never by the library.

What is computed, in the paper's notation:
  * basis phi_i = P1 hat functions on interior (non-Dirichlet) nodes, so the
    discrete space lies in H^1_0 (Section 2.2);
  * mass matrix      B_ij = int phi_i phi_j            (exact: |K|(1+d_ab)/20)
  * stiffness matrix L_ij = int grad phi_i . grad phi_j (exact: |K| g_a . g_b)
  * potential matrix (M_V)_ij = int V phi_i phi_j, by the 4-point degree-2
    rule on each tetrahedron (reading: the paper does not name a rule; one
    rule is used for every potential term and for the density so that the
    discrete energy and its gradient are consistent);
  * H = L/2 + M_ext for the fixed (linear) problem (eq. hamiltonian with the
    density-dependent terms left out).

CSR convention: rows and columns are interior DOFs numbered in node order,
columns sorted ascending within a row, the diagonal included.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# 4-point degree-2 rule on a tetrahedron: barycentric (a,b,b,b) and its
# permutations, equal weights |K|/4.
QA = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
QB = (5.0 - math.sqrt(5.0)) / 20.0
BARY = np.full((4, 4), QB)
np.fill_diagonal(BARY, QA)       # BARY[q, a] = lambda_a at quadrature point q


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volumes |K| and barycentric gradients g[K, a, :] of every tetrahedron."""
    v = xyz[tets]                                   # [nt, 4, 3]
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    vol = np.abs(det) / 6.0
    Jinv = np.linalg.inv(J)                         # lambda_{1..3} = Jinv (x - v0)
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return vol, g


def quad_points(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Physical coordinates of the 4 quadrature points of each element [nt,4,3]."""
    v = xyz[tets]
    return np.einsum("qa,kad->kqd", BARY, v)


def external_potential(xq: np.ndarray, Z: np.ndarray, R: np.ndarray) -> np.ndarray:
    """V_ext(r) = -sum_j Z_j / |r - R_j|  (eq. ext)."""
    V = np.zeros(xq.shape[:-1])
    for zj, rj in zip(Z, R):
        V -= zj / np.linalg.norm(xq - rj, axis=-1)
    return V


def dof_numbering(dirichlet: np.ndarray) -> np.ndarray:
    """dof[node] = index among interior nodes in node order, -1 on the boundary."""
    interior = dirichlet == 0
    dof = np.full(dirichlet.shape[0], -1, dtype=np.int64)
    dof[interior] = np.arange(int(interior.sum()))
    return dof


@dataclass
class Discretization:
    n: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz]
    L: np.ndarray            # float64 [nnz] stiffness
    B: np.ndarray            # float64 [nnz] mass
    Mext: np.ndarray         # float64 [nnz] external-potential matrix
    dof: np.ndarray          # int64 [n_nodes]
    vol: np.ndarray          # float64 [nt]
    grads: np.ndarray        # float64 [nt,4,3]
    Vext_q: np.ndarray       # float64 [nt,4]
    entry: np.ndarray        # int64 [nt,4,4] CSR position of (a,b), -1 if not interior
    tets: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def csr(self, vals: np.ndarray) -> sp.csr_matrix:
        return sp.csr_matrix((vals, self.col, self.row_ptr), shape=(self.n, self.n))

    @property
    def H(self) -> np.ndarray:
        return 0.5 * self.L + self.Mext

    def potential_matrix(self, Vq: np.ndarray) -> np.ndarray:
        """CSR values of (M_V)_ij = sum_K sum_q |K|/4 V(q) lambda_a(q) lambda_b(q)."""
        w = self.vol[:, None] / 4.0 * Vq                       # [nt, 4]
        loc = np.einsum("kq,qa,qb->kab", w, BARY, BARY)        # [nt, 4, 4]
        return self._scatter(loc)

    def _scatter(self, loc: np.ndarray) -> np.ndarray:
        e = self.entry.ravel()
        m = e >= 0
        return np.bincount(e[m], weights=loc.ravel()[m], minlength=self.nnz)


def csr_pattern(tets: np.ndarray, dof: np.ndarray, n: int):
    """Sorted-column CSR pattern of the P1 matrices over interior DOFs, and the
    CSR position of every element entry (a, b)."""
    d = dof[tets]                                         # [nt, 4]
    r = np.repeat(d[:, :, None], 4, axis=2)               # row dof of (a, b)
    c = np.repeat(d[:, None, :], 4, axis=1)               # col dof of (a, b)
    valid = (r >= 0) & (c >= 0)
    keys = np.where(valid, r * n + c, -1).ravel()
    good = keys >= 0
    uniq, inv = np.unique(keys[good], return_inverse=True)
    rows = uniq // n
    cols = (uniq % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    entry = np.full(keys.shape[0], -1, dtype=np.int64)
    entry[good] = inv
    return row_ptr, cols, entry.reshape(tets.shape[0], 4, 4)


def discretize(mesh, Z: np.ndarray, R: np.ndarray) -> Discretization:
    """Assemble L, B and M_ext on the interior DOFs of a mesh."""
    xyz, tets = mesh.xyz, mesh.tets.astype(np.int64)
    dof = dof_numbering(mesh.dirichlet)
    n = int((dof >= 0).sum())
    vol, g = tet_geometry(xyz, tets)
    row_ptr, col, entry = csr_pattern(tets, dof, n)
    Kloc = vol[:, None, None] * np.einsum("kad,kbd->kab", g, g)
    Mloc = vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0
    disc = Discretization(n=n, row_ptr=row_ptr, col=col, L=None, B=None, Mext=None, dof=dof,
                          vol=vol, grads=g, Vext_q=None, entry=entry, tets=tets)
    disc.L = disc._scatter(Kloc)
    disc.B = disc._scatter(Mloc)
    disc.Vext_q = external_potential(quad_points(xyz, tets), Z, R)
    disc.Mext = disc.potential_matrix(disc.Vext_q)
    return disc


def local_rows(mesh, Z: np.ndarray, R: np.ndarray, rows) -> dict:
    """Rows of L, B and M_ext for the given interior DOFs, assembled from the
    tetrahedra that touch them only, with the element formulas of discretize
    (and, the tetrahedra taken in mesh order, the same summation order).  For
    checks at sizes where assembling everything here would take too long.
    Returns {row: (cols ascending, L, B, Mext)}."""
    xyz = mesh.xyz
    dof = dof_numbering(mesh.dirichlet)
    n = int((dof >= 0).sum())
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    nodes = np.flatnonzero(np.isin(dof, rows))
    tets = mesh.tets[np.isin(mesh.tets, nodes).any(axis=1)].astype(np.int64)
    vol, g = tet_geometry(xyz, tets)
    Kloc = vol[:, None, None] * np.einsum("kad,kbd->kab", g, g)
    Mloc = np.broadcast_to(vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0, Kloc.shape)
    w = vol[:, None] / 4.0 * external_potential(quad_points(xyz, tets), Z, R)
    Vloc = np.einsum("kq,qa,qb->kab", w, BARY, BARY)
    d = dof[tets]
    r = np.repeat(d[:, :, None], 4, axis=2).ravel()
    c = np.repeat(d[:, None, :], 4, axis=1).ravel()
    keep = np.isin(r, rows) & (c >= 0)
    keys = r[keep] * n + c[keep]
    uk, inv = np.unique(keys, return_inverse=True)
    vals = [np.bincount(inv, weights=v.ravel()[keep], minlength=len(uk)) for v in (Kloc, Mloc, Vloc)]
    out = {}
    ur = uk // n
    for i in rows:
        m = ur == i
        out[int(i)] = (uk[m] % n, vals[0][m], vals[1][m], vals[2][m])
    return out


def nuclear_repulsion(Z: np.ndarray, R: np.ndarray) -> float:
    """E_nuc = sum_{j<k} Z_j Z_k / |R_j - R_k|  (Section 2.1)."""
    e = 0.0
    for j in range(len(Z)):
        for k in range(j + 1, len(Z)):
            e += Z[j] * Z[k] / float(np.linalg.norm(R[j] - R[k]))
    return e
