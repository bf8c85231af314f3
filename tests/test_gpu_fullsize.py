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
