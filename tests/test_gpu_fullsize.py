"""GPU parity at the full size of the benchmark workload (24-nucleus cluster,
n ~ 2e6 interior DOFs, p = 128), through the same launchers the benchmark
times.  The oracle is affordable here for the mesh, the CSR pattern, the
products and the preconditioner apply; the iteration itself is checked at
small sizes in test_gpu_parity.py.

Tolerances as there: indexing bit-exact, FP64 kernels 1e-12 (products, Gram)
and 1e-11 (ten CG steps) relative to the largest entry."""
import numpy as np
import pytest

import workloads as wl
from oracle import fem, native, pcal

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def c3():
    print("[gpu] full size: workload and oracle discretization", flush=True)
    w = wl.make_workload("c3", seed=0)
    d = fem.discretize(w.mesh, w.Z, w.R)
    from paper_2007_14228_amd import Solver
    s = Solver()
    s.load_workload(w)
    return w, d, s


def test_full_size_csr_is_bit_exact(c3):
    w, d, s = c3
    print(f"[gpu] full size CSR n={d.n}", flush=True)
    g = s.csr_get()
    assert np.array_equal(g["row_ptr"], d.row_ptr)
    assert np.array_equal(g["col"], d.col)
    assert _relerr(g["L"], d.L) < 1e-12
    assert _relerr(g["B"], d.B) < 1e-12
    assert _relerr(g["H"], d.H) < 1e-12


@pytest.mark.parametrize("mode", ["gather", "halo"])
def test_full_size_products_and_gram(mode, c3):
    import torch
    w, d, s = c3
    print(f"[gpu] full size SpMM ({mode}) and Gram p=128", flush=True)
    s.set_params(spmm_mode=mode)
    X = wl.random_block(77, d.n, w.p)
    Xd = _dev(X)
    HXd, BXd = s.spmm(Xd)
    rows = np.sort(np.random.default_rng(5).choice(d.n, 2000, replace=False))
    idx = torch.from_numpy(rows).to("cuda")
    HXs = HXd.index_select(0, idx).cpu().numpy()
    BXs = BXd.index_select(0, idx).cpu().numpy()
    # the oracle's rows one by one (sparse row slices times X)
    assert _relerr(HXs, d.csr(d.H)[rows] @ X) < 1e-12
    assert _relerr(BXs, d.csr(d.B)[rows] @ X) < 1e-12
    S, L0 = s.gram(Xd, HXd, BXd)
    BX = native.spmm(d.row_ptr, d.col, d.B, X)
    HX = native.spmm(d.row_ptr, d.col, d.H, X)
    assert _relerr(S, X.T @ BX) < 1e-12
    assert _relerr(L0, X.T @ HX) < 1e-12


@pytest.mark.parametrize("mode", ["gather", "halo"])
def test_full_size_preconditioner(mode, c3):
    import torch
    w, d, s = c3
    print(f"[gpu] full size preconditioner ({mode}) p=128 m=10", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    rng = np.random.default_rng(9)
    G = rng.standard_normal((d.n, w.p))
    lam = -np.abs(rng.standard_normal(w.p)) * 3.0 - 0.05
    lam[7] = 0.2                                   # identity branch
    s.set_params(precond="paper", pcg_iters=10, spmm_mode=mode)
    P = s.precondition(lam, _dev(G))
    ref = pcal.precondition(prob, G, lam, pcal.Params(precond="paper", pcg_iters=10))
    rows = np.sort(rng.choice(d.n, 5000, replace=False))
    Ps = P.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().numpy()
    assert _relerr(Ps, ref[rows]) < 1e-11
    assert np.array_equal(Ps[:, 7], G[rows, 7])


@pytest.fixture(scope="module")
def c3_trajectory(c3):
    """The oracle's first two PCAL iterations at full size from the benchmark's
    start block (seed 1000): X^0 = CholGS(V), then the identity-branch step at
    k = 0 and a step through the m = 10 inner solves at k = 1."""
    w, d, s = c3
    print("[gpu] full size: oracle CholGS and two PCAL iterations", flush=True)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    V = wl.random_block(1000, d.n, w.p)
    X0 = pcal.chol_gs(prob, V)
    X2, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper",
                                               pcg_iters=10))
    rows = np.sort(np.random.default_rng(21).choice(d.n, 2000, replace=False))
    return prob, V, X0, X2, hist, rows


def _sampled(t, rows):
    import torch
    return t.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().numpy()


def test_full_size_cholgs_start(c3, c3_trajectory):
    """X^0 = V R^{-1} with R^T R = V^T B V (Section 4.2), through the MFMA
    row-GEMM's multi-tile persistent loop (n = 2e6 rows, p = 128)."""
    w, d, s = c3
    prob, V, X0, _, _, rows = c3_trajectory
    print("[gpu] full size CholGS p=128", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper", pcg_iters=10, spmm_mode="auto")
    s.set_x0(_dev(V), orthonormalize=True)
    assert _relerr(_sampled(s.get_x(), rows), X0[rows]) < 1e-12


@pytest.mark.parametrize("mode", ["auto", "gather"])
def test_full_size_iterations_follow_the_oracle(mode, c3, c3_trajectory):
    """Two FP64 PCAL iterations at full size (the benchmark's launch
    configuration for mode "auto": LDS-halo SpMM, MFMA Gram and row-GEMM over
    31,164 row tiles, 1024-block partial sums): kkt, fea and energy at every
    iterate, eta of both steps, and 2000 sampled rows of X^2."""
    w, d, s = c3
    prob, V, X0, X2, hist, rows = c3_trajectory
    print(f"[gpu] full size FP64 iterations ({mode})", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper", pcg_iters=10, energy_every=1,
                 spmm_mode=mode)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, _, _ = s.step(3)
    assert len(st) == len(hist) == 3
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-10 * b.kkt, (a, b)
        assert abs(a["fea"] - b.fea) <= 1e-10 * b.fea + 1e-13, (a, b)
        assert abs(a["energy"] - b.energy) <= 1e-10 * abs(b.energy), (a, b)
    for k in (1, 2):
        assert abs(st[k - 1]["eta"] - hist[k].eta) <= 1e-9 * hist[k].eta
    assert _relerr(_sampled(s.get_x(), rows), X2[rows]) < 1e-10


def test_full_size_rayleigh_ritz(c3, c3_trajectory):
    """Post-processing (Section 4.3) of the full-size iterate X^2: the Ritz
    values of (Lambda0, S) at p = 128, and the rotated block X Y through the
    MFMA row-GEMM on sampled rows (columns compared up to sign, where the
    Ritz value is separated from its neighbours)."""
    w, d, s = c3
    prob, V, X0, X2, hist, rows = c3_trajectory
    print("[gpu] full size Rayleigh-Ritz p=128", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper", pcg_iters=10, energy_every=1,
                 spmm_mode="auto")
    s.set_x0(_dev(X0), orthonormalize=False)
    s.step(3)
    eig = s.postprocess()
    lam, XY = pcal.rayleigh_ritz(prob, X2)
    assert np.abs(eig - lam).max() <= 1e-10 * np.abs(lam).max()
    got = _sampled(s.get_x(), rows)
    ref = XY[rows]
    gap = np.minimum(np.diff(lam, prepend=-np.inf), np.diff(lam, append=np.inf))
    cols = np.nonzero(gap > 1e-3 * np.abs(lam).max())[0]
    assert len(cols) > w.p // 2
    sign = np.sign(np.sum(got[:, cols] * ref[:, cols], axis=0))
    assert _relerr(got[:, cols] * sign, ref[:, cols]) < 1e-8


def test_full_size_fp32_iterations_stay_close_to_the_oracle(c3, c3_trajectory):
    """The precision form's FP32 blocks at full size against the FP64 oracle:
    kkt to 1e-4, energy to 1e-5, sampled rows of X^2 to 1e-4."""
    w, d, s = c3
    prob, V, X0, X2, hist, rows = c3_trajectory
    print("[gpu] full size FP32 iterations", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=2, precond="paper", pcg_iters=10, energy_every=1,
                 spmm_mode="auto", precision="f32", refine_tol=0.0)
    s.set_x0(_dev(X0), orthonormalize=False)
    st, _, _ = s.step(3)
    assert all(a["precision"] == 1 for a in st)
    for a, b in zip(st, hist):
        assert abs(a["kkt"] - b.kkt) <= 1e-4 * b.kkt, (a, b)
        assert abs(a["energy"] - b.energy) <= 1e-5 * abs(b.energy), (a, b)
    assert _relerr(_sampled(s.get_x(), rows), X2[rows]) < 1e-4
    s.set_params(precision="f64")
