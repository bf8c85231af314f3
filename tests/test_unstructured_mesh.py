"""Unstructured graded meshes (the mesh-size law of Section 4.2, eq.
meshsizefunction, in 3-D distance; Delaunay tetrahedra) and the oracle's
discretization (Section 2.2) on them, against closed forms.

Kuhn grids have six congruent tetrahedron shapes; these meshes have
arbitrary ones, so a mistake in the per-tetrahedron gradients or quadrature
that the regular shapes hide shows here: the P1 patch test, exact mass
integrals and the variational bounds of the hydrogen spectrum."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as wl
from oracle import fem

HALF = 4.0


@pytest.fixture(scope="module")
def mesh():
    Z = np.array([6.0, 1.0])
    R = np.array([[0.3, -0.2, 0.1], [-1.1, 0.9, 0.4]])
    return wl.unstructured_mesh(HALF, Z, R, gamma1=0.6, gamma2=1.0, hmin=0.1, seed=1), Z, R


def test_delaunay_mesh_is_a_conforming_partition_of_the_box(mesh):
    m, _, _ = mesh
    vol, _ = fem.tet_geometry(m.xyz, m.tets.astype(np.int64))
    assert np.all(vol > 0)
    assert math.isclose(vol.sum(), (2 * HALF) ** 3, rel_tol=1e-12)
    faces = np.sort(m.tets[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
    uf, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(np.unique(counts)) <= {1, 2}
    # faces of one tetrahedron lie in a face of the box and tile its surface
    bf = uf[counts == 1]
    assert np.all(m.dirichlet[bf] == 1)
    P = m.xyz[bf]
    on_plane = np.zeros(len(bf), dtype=bool)
    for d in range(3):
        for s in (-HALF, HALF):
            on_plane |= np.all(P[:, :, d] == s, axis=1)
    assert on_plane.all()
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1).sum()
    assert math.isclose(area, 6 * (2 * HALF) ** 2, rel_tol=1e-12)
    # Dirichlet nodes are exactly the nodes on the box faces
    assert np.array_equal(m.dirichlet == 1, (np.abs(m.xyz) == HALF).any(axis=1))


def test_mesh_follows_the_size_law_and_has_no_slivers(mesh):
    m, Z, R = mesh
    assert wl.tet_quality(m.xyz, m.tets).min() >= 0.02
    v = m.xyz[m.tets]
    longest = np.stack([np.linalg.norm(v[:, a] - v[:, b], axis=1)
                        for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))], axis=1).max(axis=1)
    c = v.mean(axis=1)
    h = np.full(len(c), 1.0)
    for Rj, Zj in zip(R, Z):
        h = np.minimum(h, 0.6 * Zj ** -0.4 * np.linalg.norm(c - Rj, axis=1) ** 1.2)
    h = np.clip(h, 0.1, 1.0)
    # octree cubes have edge <= h; a Delaunay edge spans at most a few of them
    assert np.all(longest <= 3.5 * h)
    near = np.linalg.norm(c - R[0], axis=1) < 0.5
    far = np.linalg.norm(c - R[0], axis=1) > 3.0
    assert longest[near].max() < 0.5 * np.median(longest[far])


def test_device_capacity_of_the_pattern():
    """A 4e4-node mesh of the SCF kind stays within the device assembly's
    bounds (at most 128 tetrahedra per node, 64 entries per row)."""
    w = wl.make_workload("u2", target_dofs=40_000)
    m = w.mesh
    assert abs(m.n_dofs - 40_000) < 2_000
    assert np.bincount(m.tets.ravel()).max() <= 128
    d = fem.discretize(m, w.Z, w.R)
    assert np.diff(d.row_ptr).max() <= 64
    rows = np.repeat(np.arange(d.n), np.diff(d.row_ptr))
    assert np.all(np.diff(d.col)[np.diff(rows) == 0] > 0)
    assert int(np.sum(d.col == rows)) == d.n


def test_patch_test_and_exact_mass_integrals(mesh):
    m, Z, R = mesh
    full = wl.Mesh(m.xyz, m.tets, np.zeros_like(m.dirichlet), m.cells)
    d = fem.discretize(full, Z, R)
    Bm, Lm = d.csr(d.B), d.csr(d.L)
    ones = np.ones(d.n)
    assert math.isclose(ones @ (Bm @ ones), (2 * HALF) ** 3, rel_tol=1e-12)
    assert np.abs(Lm @ ones).max() < 1e-11
    x = m.xyz
    aff = 0.7 * x[:, 0] - 1.3 * x[:, 1] + 0.4 * x[:, 2] + 2.0
    interior = m.dirichlet == 0
    assert np.abs((Lm @ aff)[interior]).max() < 1e-10
    vol = (2 * HALF) ** 3
    assert math.isclose(x[:, 1] @ (Lm @ x[:, 1]), vol, rel_tol=1e-12)
    assert abs(x[:, 0] @ (Lm @ x[:, 2])) < 1e-10 * vol
    # int y^2 and int (x + 1/2)(x - 2z) over the box (odd terms vanish)
    ex = vol * HALF ** 2 / 3.0
    assert math.isclose(x[:, 1] @ (Bm @ x[:, 1]), ex, rel_tol=1e-12)
    assert math.isclose((x[:, 0] + 0.5) @ (Bm @ (x[:, 0] - 2.0 * x[:, 2])), ex, rel_tol=1e-12)


def test_hydrogen_levels_converge_from_above():
    """-1/2 and -1/8 Ha (1s and 2s of Z = 1): the P1 Ritz values on nested
    refinements of the size law stay above them and approach them."""
    Z = np.array([1.0])
    R = np.array([[0.13, -0.21, 0.07]])
    err1, err2 = [], []
    for g1 in (1.2, 0.6, 0.35):
        m = wl.unstructured_mesh(10.0, Z, R, g1, 2.0, 0.02, seed=3)
        d = fem.discretize(m, Z, R)
        lam = np.sort(sla.eigsh(d.csr(d.H), k=2, M=d.csr(d.B), sigma=-1.0, which="LM")[0])
        err1.append(lam[0] + 0.5)
        err2.append(lam[1] + 0.125)
    assert all(e > 0 for e in err1 + err2)
    assert err1[0] > err1[1] > err1[2] and err2[0] > err2[1] > err2[2]
    assert err1[2] < 0.02 and err2[2] < 0.015
