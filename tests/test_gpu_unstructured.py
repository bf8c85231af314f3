"""GPU parity on unstructured graded Delaunay meshes (the mesh-size law of
Section 4.2 in 3-D distance): irregular rows (7 to ~30 entries), arbitrary
tetrahedron shapes, and a halo plan whose blocks shrink where 16 rows'
neighbourhoods outgrow the LDS halo.

Tolerances as for the tensor-graded grids: CSR pattern bit-exact, values and
single products 1e-12 relative, FP64 iterations 1e-10 on kkt, converged
eigenvalue sums 1e-9 relative; the mixed-precision form within 1e-6 Ha."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as wl
from oracle import fem, native, pcal, scf

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _solver(w):
    from paper_2007_14228_amd import Solver
    s = Solver()
    s.load_workload(w)
    return s


@pytest.fixture(scope="module")
def u3s():
    w = wl.make_workload("u3", target_dofs=40_000, p=16)
    return w, fem.discretize(w.mesh, w.Z, w.R)


@pytest.fixture(scope="module")
def u2s():
    w = wl.make_workload("u2", target_dofs=15_000)
    return w, fem.discretize(w.mesh, w.Z, w.R)


@pytest.mark.parametrize("which", ["u3s", "u2s"])
def test_device_assembly_on_delaunay_meshes(which, request):
    w, d = request.getfixturevalue(which)
    print(f"[gpu] unstructured csr {which} n={d.n} nnz={d.nnz}", flush=True)
    s = _solver(w)
    g = s.csr_get()
    assert np.array_equal(g["row_ptr"], d.row_ptr)
    assert np.array_equal(g["col"], d.col)
    for k, ref in (("L", d.L), ("B", d.B), ("H", d.H)):
        assert _relerr(g[k], ref) < 1e-12, k
    s.close()


@pytest.mark.parametrize("mode", ["gather", "halo"])
@pytest.mark.parametrize("p", [16, 130])
def test_products_on_irregular_rows(p, mode, u3s):
    w, d = u3s
    print(f"[gpu] unstructured spmm/precondition p={p} {mode}", flush=True)
    s = _solver(w)
    s.set_params(spmm_mode=mode, precond="paper", pcg_iters=10)
    rng = np.random.default_rng(p)
    X = rng.standard_normal((d.n, p))
    HX, BX = s.spmm(_dev(X))
    assert _relerr(HX.cpu().numpy(), native.spmm(d.row_ptr, d.col, d.H, X)) < 1e-12
    assert _relerr(BX.cpu().numpy(), native.spmm(d.row_ptr, d.col, d.B, X)) < 1e-12
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    lam = -np.abs(rng.standard_normal(p)) - 0.1
    lam[1] = 0.5
    P = s.precondition(lam, _dev(X)).cpu().numpy()
    ref = pcal.precondition(prob, X, lam, pcal.Params(precond="paper", pcg_iters=10))
    assert _relerr(P, ref) < 1e-11
    s.close()


def test_linear_iterations_follow_the_oracle_and_converge(u3s):
    """24 nuclei, n ~ 4e4, p = 16: the first FP64 iterations against the
    oracle's, then FP64 and mixed precision to convergence against the 16
    lowest generalized eigenvalues of (H, B) from a shift-invert Lanczos
    solve."""
    w, d = u3s
    print(f"[gpu] unstructured pcal n={d.n}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(5, d.n, w.p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=4, precond="paper"))
    s = _solver(w)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=4, precond="paper", pcg_iters=10, energy_every=1)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, _, _ = s.step(5)
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-11 * abs(b.energy)
    Hm, Bm = d.csr(d.H), d.csr(d.B)
    lam = np.sort(sla.eigsh(Hm, k=w.p, M=Bm, sigma=-60.0, which="LM", tol=1e-13)[0])
    ref = float(lam.sum())
    s.set_params(beta=w.beta, tol=1e-10, max_iter=4000, precond="paper", pcg_iters=10)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, done, _ = s.step(4000)
    assert done and st[-1]["rel"] < 1e-10
    assert abs(st[-1]["energy"] - ref) <= 1e-9 * abs(ref)
    ev = s.postprocess()
    assert np.abs(np.sort(ev) - lam).max() <= 1e-8 * np.abs(lam).max()
    s.set_params(beta=w.beta, tol=1e-10, max_iter=4000, precond="paper", pcg_iters=10, precision="f32",
                 refine_tol=1e-4)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, done, _ = s.step(4000)
    assert done and st[-1]["precision"] == 0
    assert abs(st[-1]["energy"] - ref) < 1e-6
    s.close()


def test_scf_iterations_follow_the_oracle(u2s):
    """The full Kohn-Sham LDA problem on a 4-nucleus Delaunay mesh: density,
    Hartree solve and H re-assembly on irregular tetrahedra, first
    iterations against the oracle's."""
    w, d = u2s
    print(f"[gpu] unstructured scf n={d.n} p={w.p}", flush=True)
    prob = scf.KSProblem(d, w.Z, w.R)
    X0 = pcal.chol_gs(prob, wl.random_block(6, d.n, w.p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=3, precond="paper"))
    s = _solver(w)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=3, precond="paper", pcg_iters=10, scf=1, energy_every=1)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, _, _ = s.step(4)
    assert len(st) == len(hist) == 4
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-9 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-10 * abs(b.energy)
    s.close()
