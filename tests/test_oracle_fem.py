"""Pins of the oracle's discretization (Section 2.2) against closed forms."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import fem, native


def _full(mesh):
    """Same mesh with no Dirichlet nodes, so every node is a DOF."""
    return wl.Mesh(mesh.xyz, mesh.tets, np.zeros_like(mesh.dirichlet), mesh.cells)


@pytest.fixture(scope="module")
def graded():
    Z = np.array([6.0, 1.0])
    R = np.array([[0.3, -0.2, 0.1], [-1.1, 0.9, 0.4]])
    mesh = wl.graded_mesh(4.0, Z, R, gamma1=0.6, gamma2=1.0, hmin=0.1)
    return mesh, Z, R


def test_kuhn_mesh_is_a_conforming_partition(graded):
    mesh, _, _ = graded
    vol, _ = fem.tet_geometry(mesh.xyz, mesh.tets.astype(np.int64))
    assert np.all(vol > 0)
    assert math.isclose(vol.sum(), 8.0 ** 3, rel_tol=1e-12)
    # every interior face is shared by exactly two tetrahedra, boundary faces by one
    faces = np.sort(mesh.tets[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(np.unique(counts)) <= {1, 2}
    nx, ny, nz = mesh.cells
    n_boundary_faces = 4 * (nx * ny + ny * nz + nx * nz)     # 2 triangles per boundary quad
    assert int((counts == 1).sum()) == n_boundary_faces


def test_c1_sizes():
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    assert w.mesh.n_nodes == 17 ** 3
    assert d.n == 15 ** 3
    # 15 stencil points per node of a Kuhn grid (itself, 6 axis, 6 face-diagonal,
    # 2 body-diagonal), truncated at the Dirichlet boundary: count pairs (i, i+v)
    # for the 7 positive offsets v of the stencil and double them.
    offsets = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)]
    pairs = sum(np.prod([15 - o for o in v]) for v in offsets)
    assert d.nnz == 15 ** 3 + 2 * pairs == 45403
    rows = np.repeat(np.arange(d.n), np.diff(d.row_ptr))
    assert np.all(np.diff(d.col)[np.diff(rows) == 0] > 0)      # sorted, unique in a row
    assert int(np.sum(d.col == rows)) == d.n                     # diagonal in every row


def test_mass_and_stiffness_closed_forms(graded):
    mesh, Z, R = graded
    d = fem.discretize(_full(mesh), Z, R)
    Bm = d.csr(d.B)
    Lm = d.csr(d.L)
    ones = np.ones(d.n)
    # sum_ij B_ij = |Omega|, and L annihilates constants and affine functions
    assert math.isclose(ones @ (Bm @ ones), 8.0 ** 3, rel_tol=1e-12)
    assert np.abs(Lm @ ones).max() < 1e-12
    x = mesh.xyz
    aff = 0.7 * x[:, 0] - 1.3 * x[:, 1] + 0.4 * x[:, 2] + 2.0
    interior = mesh.dirichlet == 0
    assert np.abs((Lm @ aff)[interior]).max() < 1e-11
    # B integrates the product of two affine functions exactly (degree 2)
    u = x[:, 0] + 0.5
    v = x[:, 0] - 2.0 * x[:, 2]
    # int_{[-4,4]^3} (x + 1/2)(x - 2z) = int x^2 = 64 * 2 * 4^3 / 3 (odd terms vanish)
    assert math.isclose(u @ (Bm @ v), 64.0 * (2 * 4.0 ** 3 / 3.0), rel_tol=1e-12)
    exact2 = 64.0 * (2 * 4.0 ** 3 / 3.0)          # int x^2 over the cube
    assert math.isclose(x[:, 0] @ (Bm @ x[:, 0]), exact2, rel_tol=1e-12)
    # x^T L x = int |grad x|^2 = |Omega|
    assert math.isclose(x[:, 0] @ (Lm @ x[:, 0]), 8.0 ** 3, rel_tol=1e-12)


def test_quadrature_rule_reproduces_mass_and_degree_two(graded):
    mesh, Z, R = graded
    d = fem.discretize(mesh, Z, R)
    # M(V = 1) is the consistent mass matrix: the rule is exact for degree 2
    assert np.allclose(d.potential_matrix(np.ones_like(d.Vext_q)), d.B, rtol=1e-13, atol=1e-15)
    # the rule integrates x*y exactly over the whole box
    xq = fem.quad_points(mesh.xyz, mesh.tets.astype(np.int64))
    f = xq[..., 0] * xq[..., 1] + xq[..., 2] ** 2
    val = float(np.sum(d.vol[:, None] / 4.0 * f))
    assert math.isclose(val, 64.0 * (2 * 4.0 ** 3 / 3.0), rel_tol=1e-12)
    assert np.all(np.isfinite(d.Vext_q)) and np.all(d.Vext_q < 0)


def test_poisson_manufactured_solution_second_order():
    """-Laplace u = f on [0,1]^3, u = sin(pi x) sin(pi y) sin(pi z): nodal error O(h^2)."""
    errs = []
    for c in (8, 16):
        ax = wl.uniform_axis(0.0, 1.0, c)
        mesh = wl.kuhn_mesh(ax, ax, ax)
        d = fem.discretize(mesh, np.zeros(0), np.zeros((0, 3)))
        xq = fem.quad_points(mesh.xyz, mesh.tets.astype(np.int64))
        fq = 3 * math.pi ** 2 * np.prod(np.sin(math.pi * xq), axis=-1)
        w = d.vol[:, None] / 4.0 * fq
        loc = w @ fem.BARY
        dv = d.dof[d.tets].ravel()
        m = dv >= 0
        b = np.bincount(dv[m], weights=loc.ravel()[m], minlength=d.n)
        U = sp.linalg.spsolve(d.csr(d.L).tocsc(), b)
        xin = mesh.xyz[mesh.dirichlet == 0]
        errs.append(np.abs(U - np.prod(np.sin(math.pi * xin), axis=-1)).max())
    assert 3.3 < errs[0] / errs[1] < 5.0


def test_particle_in_a_box_eigenvalue_second_order():
    """-1/2 Laplace on [0,1]^3: lambda_1 = 3 pi^2 / 2; P1 error is O(h^2) from above."""
    exact = 1.5 * math.pi ** 2
    errs = []
    for c in (6, 12):
        ax = wl.uniform_axis(0.0, 1.0, c)
        mesh = wl.kuhn_mesh(ax, ax, ax)
        d = fem.discretize(mesh, np.zeros(0), np.zeros((0, 3)))
        lam = sla.eigh(d.csr(0.5 * d.L).toarray(), d.csr(d.B).toarray(), eigvals_only=True,
                       subset_by_index=[0, 0])[0]
        assert lam > exact
        errs.append(lam - exact)
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_native_spmm_matches_scipy(graded):
    mesh, Z, R = graded
    d = fem.discretize(mesh, Z, R)
    X = np.random.default_rng(3).standard_normal((d.n, 5))
    ref = d.csr(d.H) @ X
    assert np.allclose(native.spmm(d.row_ptr, d.col, d.H, X), ref, rtol=1e-13, atol=1e-13)
    lam = np.array([-1.0, -0.5, 0.0, 0.25, -3.0])
    Ys = native.shifted_spmm(d.row_ptr, d.col, 0.5 * d.L, d.B, lam, X)
    for l in range(5):
        refl = d.csr(0.5 * d.L - lam[l] * d.B) @ X[:, l]
        assert np.allclose(Ys[:, l], refl, rtol=1e-13, atol=1e-13)


def test_nuclear_repulsion_closed_form():
    Z = np.array([1.0, 8.0, 6.0])
    R = np.array([[0.0, 0, 0], [2.0, 0, 0], [0, 0, 4.0]])
    assert math.isclose(fem.nuclear_repulsion(Z, R), 8 / 2 + 6 / 4 + 48 / math.sqrt(20.0),
                        rel_tol=1e-15)


def test_local_rows_equal_the_full_assembly(graded):
    """fem.local_rows (the assembly of single rows from the tetrahedra around
    them, used for sampled checks at sizes the full assembly cannot reach)
    gives the same columns and values as discretize.  Every 7th row is
    compared, which includes rows next to the boundary and rows at the
    refined nuclei.  Planted mistakes this catches (checked): a tetrahedron
    dropped from the local set, the potential term's weights |K|/4 changed."""
    mesh, Z, R = graded
    d = fem.discretize(mesh, Z, R)
    rows = np.arange(0, d.n, 7)
    loc = fem.local_rows(mesh, Z, R, rows)
    assert sorted(loc) == list(rows)
    for i in rows:
        s, e = d.row_ptr[i], d.row_ptr[i + 1]
        cols, Lv, Bv, Mv = loc[int(i)]
        assert np.array_equal(cols, d.col[s:e])
        for got, ref in ((Lv, d.L[s:e]), (Bv, d.B[s:e]), (Mv, d.Mext[s:e])):
            assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
