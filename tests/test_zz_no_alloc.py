"""ofks_gram_noalloc (the Gram for callers that cannot allocate device
memory) through the C ABI, against ofks_gram on the same inputs: two calls in
a row on one context, the second with a smaller block, then a call from a
second, smaller system on the same device (the device's scratch array keeps
the previous call's contents).  Tolerance 1e-12 relative to the largest
entry (the two entry points may split the rows differently), and the oracle's
X^T BX, X^T HX at the same bar."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import fem, native

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _both(s, X):
    """(S, L0) from ofks_gram and from ofks_gram_noalloc, called directly."""
    from paper_2007_14228_amd.solver import _dev_ptr, _np_ptr
    HX, BX = s.spmm(X)
    p = int(X.shape[1])
    out = []
    for name in ("ofks_gram", "ofks_gram_noalloc"):
        S, L0 = np.empty((p, p)), np.empty((p, p))
        rc = getattr(s.lib, name)(s.h, p, _dev_ptr(X), _dev_ptr(HX), _dev_ptr(BX), _np_ptr(S), _np_ptr(L0))
        assert rc == 0, (name, s.lib.ofks_last_error(s.h))
        out.append((S, L0))
    return out


def _oracle(d, X):
    return (X.T @ native.spmm(d.row_ptr, d.col, d.B, X), X.T @ native.spmm(d.row_ptr, d.col, d.H, X))


def test_gram_noalloc_matches_gram_on_successive_calls():
    import torch
    from paper_2007_14228_amd import Solver
    Z = np.array([6.0, 1.0, 8.0])
    R = np.array([[0.3, -0.2, 0.1], [-1.4, 0.9, 0.4], [1.1, 1.3, -0.9]])
    mesh = wl.graded_mesh(5.0, Z, R, gamma1=0.5, gamma2=1.2, hmin=0.1)
    d = fem.discretize(mesh, Z, R)
    s = Solver()
    s.mesh_load(mesh.xyz, mesh.tets, mesh.dirichlet)
    s.nuclei_set(Z, R)
    s.assemble()
    for seed, p in ((1, 130), (2, 33)):                  # the second call is smaller
        print(f"[gpu] gram_noalloc n={d.n} p={p}", flush=True)
        X = wl.random_block(seed, d.n, p)
        (S, L0), (Sn, L0n) = _both(s, torch.from_numpy(X).cuda())
        assert _relerr(Sn, S) < 1e-12 and _relerr(L0n, L0) < 1e-12
        So, Lo = _oracle(d, X)
        assert _relerr(Sn, So) < 1e-12 and _relerr(L0n, Lo) < 1e-12
    s.close()
    # a second, smaller system on the same device
    w = wl.make_workload("c1")
    d1 = fem.discretize(w.mesh, w.Z, w.R)
    s1 = Solver()
    s1.load_workload(w)
    print(f"[gpu] gram_noalloc n={d1.n} p=4", flush=True)
    X = wl.random_block(3, d1.n, 4)
    (S, L0), (Sn, L0n) = _both(s1, torch.from_numpy(X).cuda())
    assert _relerr(Sn, S) < 1e-12 and _relerr(L0n, L0) < 1e-12
    So, Lo = _oracle(d1, X)
    assert _relerr(Sn, So) < 1e-12 and _relerr(L0n, Lo) < 1e-12
    s1.close()


def test_gram_noalloc_rejects_p_beyond_its_scratch():
    import torch
    from paper_2007_14228_amd import Solver
    from paper_2007_14228_amd.solver import _np_ptr
    w = wl.make_workload("c1")
    s = Solver()
    s.load_workload(w)
    S = np.empty(1)
    X = torch.zeros((w.mesh.n_dofs, 1), dtype=torch.float64, device="cuda")
    ptr = ctypes.c_void_p(X.data_ptr())
    rc = s.lib.ofks_gram_noalloc(s.h, 1025, ptr, ptr, ptr, _np_ptr(S), _np_ptr(S))
    assert rc == -4 and b"outside" in s.lib.ofks_last_error(s.h)
    s.close()
