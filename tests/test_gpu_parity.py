"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: indexing bit-exact; FP64 single-kernel results 1e-12 relative
(summation order differs); converged energies and eigenvalues 1e-10 relative.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import fem, native, pcal, scf

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torch():
    import torch
    return torch


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _solver_for(w):
    from paper_2007_14228_amd import Solver
    s = Solver()
    s.load_workload(w)
    return s


def _relerr(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


@pytest.fixture(scope="module")
def c1():
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    return w, d


@pytest.fixture(scope="module")
def graded():
    """A graded multi-nucleus mesh: rows of different lengths, several tiles."""
    Z = np.array([6.0, 1.0, 8.0])
    R = np.array([[0.3, -0.2, 0.1], [-1.4, 0.9, 0.4], [1.1, 1.3, -0.9]])
    mesh = wl.graded_mesh(5.0, Z, R, gamma1=0.5, gamma2=1.2, hmin=0.1)
    w = wl.Workload("graded", mesh, Z, R, p=7, beta=1.0, scf=False, seed=0)
    return w, fem.discretize(mesh, Z, R)


@pytest.mark.parametrize("which", ["c1", "graded"])
def test_csr_pattern_bit_exact_and_values(which, c1, graded):
    w, d = c1 if which == "c1" else graded
    print(f"[gpu] csr parity {which} n={d.n} nnz={d.nnz}", flush=True)
    s = _solver_for(w)
    g = s.csr_get()
    assert np.array_equal(g["row_ptr"], d.row_ptr)
    assert np.array_equal(g["col"], d.col)
    assert _relerr(g["L"], d.L) < 1e-13
    assert _relerr(g["B"], d.B) < 1e-13
    assert _relerr(g["H"], d.H) < 1e-13


@pytest.mark.parametrize("mode", ["gather", "halo"])
@pytest.mark.parametrize("p", [1, 3, 4, 11, 16, 33, 64, 128, 130, 260, 512])
def test_dual_spmm(p, mode, graded):
    """Both SpMM kernels: row-gather, and LDS-halo (p = 33, 130, 260: a ragged
    last 512-byte column slice)."""
    w, d = graded
    print(f"[gpu] spmm p={p} mode={mode}", flush=True)
    s = _solver_for(w)
    s.set_params(spmm_mode=mode)
    X = np.random.default_rng(p).standard_normal((d.n, p))
    HX, BX = s.spmm(_dev(X))
    assert _relerr(_host(HX), native.spmm(d.row_ptr, d.col, d.H, X)) < 1e-12
    assert _relerr(_host(BX), native.spmm(d.row_ptr, d.col, d.B, X)) < 1e-12


@pytest.mark.parametrize("p", [1, 4, 11, 33, 128, 260, 512])
def test_gram(p, graded):
    w, d = graded
    print(f"[gpu] gram p={p}", flush=True)
    s = _solver_for(w)
    rng = np.random.default_rng(100 + p)
    X, HX, BX = (rng.standard_normal((d.n, p)) for _ in range(3))
    S, L0 = s.gram(_dev(X), _dev(HX), _dev(BX))
    assert _relerr(S, X.T @ BX) < 1e-12
    assert _relerr(L0, X.T @ HX) < 1e-12


@pytest.mark.parametrize("mode", ["gather", "halo"])
@pytest.mark.parametrize("p", [1, 5, 16, 128, 130, 512])
def test_preconditioner_cg(p, mode, graded):
    w, d = graded
    print(f"[gpu] precondition p={p} mode={mode}", flush=True)
    s = _solver_for(w)
    s.set_params(precond="paper", pcg_iters=10, spmm_mode=mode)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    rng = np.random.default_rng(7 + p)
    G = rng.standard_normal((d.n, p))
    lam = -np.abs(rng.standard_normal(p)) - 0.1
    if p > 1:
        lam[1] = 0.5                        # identity branch
    P = _host(s.precondition(lam, _dev(G)))
    ref = pcal.precondition(prob, G, lam, pcal.Params(precond="paper", pcg_iters=10))
    assert _relerr(P, ref) < 1e-11


@pytest.mark.parametrize("mode", ["gather", "halo"])
def test_products_are_bitwise_repeatable(mode, graded):
    """Fixed-order reductions: the same call twice gives the same bits (the
    dual product, and the preconditioner whose CG sums per-block partials)."""
    w, d = graded
    p = 130
    print(f"[gpu] repeatability mode={mode}", flush=True)
    s = _solver_for(w)
    s.set_params(precond="paper", pcg_iters=10, spmm_mode=mode)
    rng = np.random.default_rng(21)
    X = _dev(rng.standard_normal((d.n, p)))
    lam = -np.abs(rng.standard_normal(p)) - 0.1
    a = [_host(t) for t in s.spmm(X)] + [_host(s.precondition(lam, X))]
    b = [_host(t) for t in s.spmm(X)] + [_host(s.precondition(lam, X))]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_matrix_without_halo_plan_uses_row_gather():
    """csr_load of a pattern with a row wider than the LDS halo: no halo plan,
    the automatic choice takes the row-gather kernel, a forced halo kernel is
    an error."""
    import scipy.sparse as sp
    from paper_2007_14228_amd import Solver
    print("[gpu] csr_load wide row", flush=True)
    n, p = 300, 64
    rng = np.random.default_rng(4)
    A = sp.diags([np.ones(n - 1), 4.0 * np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="lil")
    A[1, :250] = rng.standard_normal(250)
    A[1, 1] = 5.0
    A = A.tocsr()
    A.sort_indices()
    rp, col = A.indptr.astype(np.int64), A.indices.astype(np.int32)
    H, B = A.data.copy(), np.abs(A.data) + 1.0
    s = Solver()
    s.csr_load(_dev(rp), _dev(col), _dev(H), _dev(B), _dev(0.5 * H))
    X = rng.standard_normal((n, p))
    HX, BX = s.spmm(_dev(X))
    Bm = sp.csr_matrix((B, col, rp), shape=(n, n))
    assert _relerr(_host(HX), A @ X) < 1e-12
    assert _relerr(_host(BX), Bm @ X) < 1e-12
    s.set_params(spmm_mode="halo")
    with pytest.raises(RuntimeError):
        s.spmm(_dev(X))


@pytest.mark.parametrize("mode", ["gather", "halo"])
def test_step_parity_in_both_spmm_modes(mode, c1):
    """Three FP64 iterations with the paper preconditioner at p = 72 (two
    column slices, the second ragged) through each SpMM kernel."""
    w, d = c1
    p = 72
    print(f"[gpu] step parity c1 p={p} mode={mode}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(8, d.n, p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=3, precond="paper"))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 3, beta=w.beta, tol=1e-30, precond="paper", pcg_iters=10, energy_every=1,
                  spmm_mode=mode)
    assert len(st) == len(hist) == 4
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-11 * abs(b.energy)


def _run_gpu(s, X0, max_iter, **params):
    s.set_params(max_iter=max_iter, **params)
    s.set_x0(_dev(X0), orthonormalize=False)
    stats, done, rc = s.step(max_iter + 1)
    return stats


@pytest.mark.parametrize("precond", ["none", "paper"])
def test_first_iterations_follow_the_oracle(precond, c1):
    """Step parity: kkt, fea, rel and eta of the first iterations from the same X0."""
    w, d = c1
    print(f"[gpu] step parity c1 {precond}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(0, d.n, w.p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=6, precond=precond))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 6, beta=w.beta, tol=1e-30, precond=precond, pcg_iters=10)
    assert len(st) == len(hist) == 7
    for a, b in zip(st, hist):
        assert a["k"] == b.k
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt
        assert abs(a["fea"] - b.fea) <= 1e-10 * b.fea + 1e-13     # fea at k = 0 is rounding noise
        assert abs(a["energy"] - b.energy) <= 1e-11 * abs(b.energy)
    # eta used for each step (oracle records it at the next iterate)
    for k in range(1, 7):
        assert abs(st[k - 1]["eta"] - hist[k].eta) <= 1e-9 * hist[k].eta


@pytest.mark.parametrize("algorithm,precond,step_rule", [("plam", "none", "bb2"), ("plam", "paper", "bb2"),
                                                         ("pcal", "paper", "bb1"), ("pcal", "paper", "abb1"),
                                                         ("pcal", "paper", "abb2"), ("pcal", "none", "fixed")])
def test_other_algorithms_and_step_rules_follow_the_oracle(algorithm, precond, step_rule, c1):
    """Algorithm PLAM and the BB1/ABB/fixed step rules (Section 4.4): the first
    iterations against the oracle's, then (PLAM) convergence to the dense
    eigenvalues."""
    w, d = c1
    print(f"[gpu] {algorithm} {precond} {step_rule}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(0, d.n, w.p))
    prm = dict(beta=w.beta, precond=precond, step_rule=step_rule, algorithm=algorithm)
    if step_rule == "fixed":
        prm["eta0"] = 40.0
    _, hist = pcal.pcal(prob, X0, pcal.Params(tol=1e-30, max_iter=6, **prm))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 6, tol=1e-30, pcg_iters=10, energy_every=1, **prm)
    assert len(st) == len(hist) == 7
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-11 * abs(b.energy)
    if algorithm == "plam":
        s.set_params(tol=1e-10, max_iter=3000, pcg_iters=10, **prm)
        s.set_x0(_dev(X0), orthonormalize=False)
        st, done, _ = s.step(3000)
        assert done and st[-1]["rel"] < 1e-10
        ref = np.array(json.load(open(os.path.join(GOLDEN, "c1_dense_eigs.json")))["eigenvalues"][: w.p])
        assert np.allclose(s.postprocess(), ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("p", [40, 128, 130, 512])
def test_first_iterations_follow_the_oracle_wide_blocks(p, c1):
    """Step parity at block widths where the row GEMM runs on the matrix cores
    (p = 130: a ragged last column tile), paper preconditioner, FP64."""
    w, d = c1
    print(f"[gpu] step parity c1 p={p}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(5, d.n, p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=3, precond="paper"))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 3, beta=w.beta, tol=1e-30, precond="paper", pcg_iters=10, energy_every=1)
    assert len(st) == len(hist) == 4
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-11 * abs(b.energy)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("precond", ["none", "paper"])
@pytest.mark.parametrize("p", [64, 128])
def test_row_gemm_widths_follow_the_oracle(p, precond, precision, c1):
    """p = 64 and 128, where the gradient row GEMM holds the multiplier in LDS
    (FP64 at p = 128 in two 128-column halves, one per block), with the plain
    gradient epilogue (no preconditioner) and the PCG-start one: the first
    iterations against the oracle's (FP64 blocks: kkt 1e-10 and energy 1e-11
    relative; FP32 blocks: 1e-4 and 1e-5)."""
    w, d = c1
    print(f"[gpu] row gemm width p={p} {precond} {precision}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(9, d.n, p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=3, precond=precond))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 3, beta=w.beta, tol=1e-30, precond=precond, pcg_iters=10, energy_every=1,
                  precision=precision)
    assert len(st) == len(hist) == 4
    assert st[0]["precision"] == (1 if precision == "f32" else 0)
    tk, te = (1e-10, 1e-11) if precision == "f64" else (1e-4, 1e-5)
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= tk * b.kkt
        assert abs(a["energy"] - b.energy) <= te * abs(b.energy)


@pytest.mark.parametrize("mode", ["gather", "halo"])
@pytest.mark.parametrize("p", [40, 130, 260, 512])
def test_fp32_iterations_stay_close_to_the_oracle(p, mode, c1):
    """The FP32 block path (FP32 matrix-core products) tracks the FP64 oracle
    over the first iterations to FP32 accuracy, through either SpMM kernel
    (halo: p = 40 and 260 end in a ragged 128-column slice of 16-byte
    segments, p = 130 takes element loads)."""
    w, d = c1
    print(f"[gpu] fp32 step c1 p={p} mode={mode}", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(6, d.n, p))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper"))
    s = _solver_for(w)
    st = _run_gpu(s, X0, 2, beta=w.beta, tol=1e-30, precond="paper", pcg_iters=10, energy_every=1,
                  precision="f32", spmm_mode=mode)
    assert st[0]["precision"] == 1
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-4 * b.kkt
        assert abs(a["energy"] - b.energy) <= 1e-5 * abs(b.energy)


@pytest.mark.parametrize("precond", ["none", "paper"])
def test_converged_eigenvalues_match_dense_lapack(precond, c1):
    w, d = c1
    print(f"[gpu] c1 converge {precond}", flush=True)
    s = _solver_for(w)
    X0 = wl.random_block(0, d.n, w.p)
    s.set_params(beta=w.beta, tol=1e-10, max_iter=2000, precond=precond)
    s.set_x0(_dev(X0), orthonormalize=True)
    stats, done, rc = s.step(2000)
    assert done and stats[-1]["rel"] < 1e-10
    eig = s.postprocess()
    ref = np.array(json.load(open(os.path.join(GOLDEN, "c1_dense_eigs.json")))["eigenvalues"][: w.p])
    assert np.allclose(eig, ref, rtol=1e-10, atol=0)
    assert stats[-1]["fea"] < 1e-9


def test_single_column_feasible_every_iterate(c1):
    w, d = c1
    print("[gpu] p=1", flush=True)
    s = _solver_for(w)
    s.set_params(beta=1.0, tol=1e-10, max_iter=1000, precond="paper")
    s.set_x0(_dev(wl.random_block(5, d.n, 1)), orthonormalize=True)
    stats, done, _ = s.step(1000)
    assert done
    assert max(x["fea"] for x in stats) < 1e-14
    ref = json.load(open(os.path.join(GOLDEN, "c1_dense_eigs.json")))["eigenvalues"][0]
    assert abs(stats[-1]["energy"] - ref) < 1e-10 * abs(ref)


def test_get_x_is_b_orthonormal_at_convergence(c1):
    w, d = c1
    s = _solver_for(w)
    s.set_params(beta=w.beta, tol=1e-10, max_iter=2000, precond="paper")
    s.set_x0(_dev(wl.random_block(3, d.n, w.p)), orthonormalize=True)
    s.step(2000)
    X = _host(s.get_x())
    S = X.T @ native.spmm(d.row_ptr, d.col, d.B, X)
    assert np.abs(S - np.eye(w.p)).max() < 1e-9


# ----------------------------------------------------------------------------
# Kohn-Sham (SCF) pieces
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def lih():
    ax = wl.uniform_axis(-6.0, 6.0, 10)
    mesh = wl.kuhn_mesh(ax, ax, ax)
    Z = np.array([3.0, 1.0])
    R = np.array([[-1.2, 0.0, 0.0], [1.2, 0.0, 0.0]])
    w = wl.Workload("lih", mesh, Z, R, p=2, beta=1.0, scf=True, seed=0)
    return w, fem.discretize(mesh, Z, R)


def test_density_xc_hartree_and_hamiltonian(lih):
    w, d = lih
    print("[gpu] build_hamiltonian", flush=True)
    prob = scf.KSProblem(d, w.Z, w.R)
    X = pcal.chol_gs(prob, wl.random_block(2, d.n, 2))
    s = _solver_for(w)
    out = s.build_hamiltonian(_dev(X))
    Hval, rho, U, parts = prob.build(X)
    assert _relerr(_host(out["rho"]), rho) < 1e-13
    from oracle.xc import lda_xc
    eps, vxc = lda_xc(rho)
    assert _relerr(_host(out["vxc"]), vxc) < 1e-12
    assert _relerr(_host(out["eps"]), eps) < 1e-12
    assert _relerr(_host(out["U"]), U) < 1e-10          # both CGs stop at 1e-12 relative residual
    assert abs(out["parts"][0] - parts["nelec"]) < 1e-12 * parts["nelec"]
    assert abs(out["parts"][1] - parts["xc"]) < 1e-12 * abs(parts["xc"])
    assert abs(out["parts"][2] - parts["int_vxc_rho"]) < 1e-12 * abs(parts["int_vxc_rho"])
    assert abs(out["parts"][3] - parts["har"]) < 1e-10 * parts["har"]
    g = s.csr_get()
    assert _relerr(g["H"], Hval) < 1e-11


def test_hartree_graph_replays_match_eager_launches(lih):
    """The Hartree CG replayed as a captured graph gives bit-identical
    potentials to eager launches, over consecutive solves (each many replays,
    with host synchronization between them)."""
    w, d = lih
    print("[gpu] hartree graph vs eager", flush=True)
    prob = scf.KSProblem(d, w.Z, w.R)
    Xs = [pcal.chol_gs(prob, wl.random_block(40 + k, d.n, 2)) for k in range(3)]
    Us = {}
    for use in (0, 1):
        s = _solver_for(w)
        s.set_params(use_graphs=use)
        Us[use] = [_host(s.build_hamiltonian(_dev(X))["U"]) for X in Xs]
    for a, b in zip(Us[0], Us[1]):
        assert np.array_equal(a, b)


def test_scf_pcal_energy_matches_the_oracle(lih):
    w, d = lih
    print("[gpu] scf pcal", flush=True)
    prob = scf.KSProblem(d, w.Z, w.R)
    X0 = pcal.chol_gs(prob, wl.random_block(0, d.n, 2))
    _, hist = pcal.pcal(prob, X0, pcal.Params(beta=1.0, tol=1e-10, max_iter=2000, precond="paper"))
    s = _solver_for(w)
    s.set_params(beta=1.0, tol=1e-10, max_iter=2000, precond="paper", scf=1)
    s.set_x0(_dev(X0), orthonormalize=False)
    stats, done, _ = s.step(2000)
    assert done and stats[-1]["rel"] < 1e-10
    E_ref = hist[-1].energy
    assert abs(stats[-1]["energy"] - E_ref) < 1e-10 * abs(E_ref)
    parts = s.energy()
    assert abs(parts[4] - E_ref) < 1e-10 * abs(E_ref)
    assert abs(parts[5] - 4.0) < 1e-9                     # 2 electrons per orbital, p = 2


# ----------------------------------------------------------------------------
# precision form
# ----------------------------------------------------------------------------

def test_mixed_precision_with_fp64_refinement(c1):
    w, d = c1
    print("[gpu] mixed c1", flush=True)
    s = _solver_for(w)
    s.set_params(beta=w.beta, tol=1e-10, max_iter=3000, precond="paper", precision="f32", refine_tol=1e-4)
    s.set_x0(_dev(wl.random_block(0, d.n, w.p)), orthonormalize=True)
    stats, done, _ = s.step(3000)
    assert done
    assert stats[0]["precision"] == 1 and stats[-1]["precision"] == 0
    ref = np.array(json.load(open(os.path.join(GOLDEN, "c1_dense_eigs.json")))["eigenvalues"][: w.p])
    assert abs(stats[-1]["energy"] - ref.sum()) < 1e-6


def test_fp32_stall_switches_to_fp64(c1):
    """An FP32 phase asked for a residual below its rounding floor stops
    improving; after 50 iterations without a new best it switches to FP64 and
    the run converges."""
    w, d = c1
    print("[gpu] fp32 stall", flush=True)
    s = _solver_for(w)
    s.set_params(beta=w.beta, tol=1e-10, max_iter=4000, precond="paper", precision="f32", refine_tol=1e-14)
    s.set_x0(_dev(wl.random_block(0, d.n, w.p)), orthonormalize=True)
    stats, done, _ = s.step(4000)
    assert done and stats[-1]["rel"] < 1e-10
    prec = [x["precision"] for x in stats]
    k64 = prec.index(0)
    assert k64 > 50 and all(q == 1 for q in prec[:k64]) and all(q == 0 for q in prec[k64:])
    ref = np.array(json.load(open(os.path.join(GOLDEN, "c1_dense_eigs.json")))["eigenvalues"][: w.p])
    assert abs(stats[-1]["energy"] - ref.sum()) < 1e-8


# ----------------------------------------------------------------------------
# errors are reported, not faulted
# ----------------------------------------------------------------------------

def test_invalid_calls_return_errors(c1):
    from paper_2007_14228_amd import OfksError, Solver
    w, d = c1
    s = Solver()
    with pytest.raises(OfksError):
        s.step(1)                                   # no system
    s.load_workload(w)
    with pytest.raises(OfksError):
        s.set_params(precond="paper", pcg_iters=0)
    s.set_params()
    with pytest.raises(ValueError):
        s.set_x0(_dev(np.zeros((d.n + 1, 2))))      # wrong row count, caught before the call
    with pytest.raises(OfksError):
        s.set_x0(_dev(np.zeros((d.n, 3))))          # V^T B V singular


def test_degenerate_inputs(c1):
    """Empty and degenerate inputs return errors, never faults; the smallest
    real system (one interior DOF, p = 1) converges to H_00 / B_00."""
    import ctypes
    from paper_2007_14228_amd import OfksError, Solver
    w, d = c1
    print("[gpu] degenerate inputs", flush=True)
    s = _solver_for(w)
    s.set_params()
    X = _dev(wl.random_block(0, d.n, 3))
    # p = 0 and p > 1024 through the C ABI directly (the binding rejects them earlier)
    assert s.lib.ofks_set_x0(s.h, 0, ctypes.c_void_p(X.data_ptr()), 1) == -1
    assert s.lib.ofks_set_x0(s.h, 1025, ctypes.c_void_p(X.data_ptr()), 1) == -1
    with pytest.raises(OfksError):
        s.step(1)                                           # no X0 yet
    # a column with zero B-norm, taken as given
    Z = wl.random_block(1, d.n, 3)
    Z[:, 1] = 0.0
    with pytest.raises(OfksError, match="zero B-norm"):
        s.set_x0(_dev(Z), orthonormalize=False)
    # a mesh without interior nodes
    ax = wl.uniform_axis(0.0, 1.0, 1)
    s0 = Solver()
    with pytest.raises(OfksError, match="no interior"):
        s0.load_workload(wl.Workload("empty", wl.kuhn_mesh(ax, ax, ax), np.array([1.0]),
                                     np.array([[0.5, 0.5, 0.5]]), p=1, beta=1.0, scf=False, seed=0))
    # one interior DOF, one column
    ax = wl.uniform_axis(-1.0, 1.0, 2)
    w1 = wl.Workload("one", wl.kuhn_mesh(ax, ax, ax), np.array([1.0]), np.array([[0.3, 0.2, 0.1]]),
                     p=1, beta=1.0, scf=False, seed=0)
    d1 = fem.discretize(w1.mesh, w1.Z, w1.R)
    assert d1.n == 1
    s1 = _solver_for(w1)
    s1.set_params(tol=1e-12, max_iter=50, precond="paper")
    s1.set_x0(_dev(np.array([[2.0]])), orthonormalize=True)
    st, done, _ = s1.step(50)
    assert done
    eig = s1.postprocess()
    assert abs(eig[0] - d1.H[0] / d1.B[0]) <= 1e-14 * abs(d1.H[0] / d1.B[0])
