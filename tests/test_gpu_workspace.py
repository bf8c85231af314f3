"""The caller-owned workspace (ofks_workspace_size / ofks_set_workspace),
through the C ABI.

For each iteration form, the run with the state carved from a workspace of
exactly the size ofks_workspace_size reports must equal the run with library
allocation bit for bit (same kernels, same reduction order), while the
device's free memory does not fall (no hipMalloc inside set_x0 or step).  A
workspace one 256-byte piece short fails with ECAPACITY, never a fault."""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
FIELDS = ("k", "precond_used", "precision", "fell_back", "energy", "kkt", "fea", "rel", "eta")


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _same(a, b):
    return a == b or (isinstance(a, float) and math.isnan(a) and math.isnan(b))


def _lih():
    ax = wl.uniform_axis(-6.0, 6.0, 10)
    mesh = wl.kuhn_mesh(ax, ax, ax)
    return wl.Workload("lih", mesh, np.array([3.0, 1.0]), np.array([[-1.2, 0.0, 0.0], [1.2, 0.0, 0.0]]),
                       p=2, beta=1.0, scf=True, seed=0)


CASES = {
    "fp64": dict(wk="c1", params=dict(precond="paper"), steps=25),
    "mixed": dict(wk="c1", params=dict(precond="paper", precision="f32", refine_tol=0.1), steps=70),
    "scf": dict(wk="lih", params=dict(precond="paper", scf=1), steps=15),
    "graph": dict(wk="c1", params=dict(precond="graph", fallback_stall=6), steps=30),
}


@pytest.mark.parametrize("case", list(CASES))
def test_workspace_run_equals_library_run(case):
    import torch
    from oracle import gnn
    from paper_2007_14228_amd import Solver
    cfg = CASES[case]
    w = wl.make_workload("c1") if cfg["wk"] == "c1" else _lih()
    print(f"[gpu] workspace {case}", flush=True)
    prm = dict(beta=w.beta, tol=1e-30, max_iter=500, pcg_iters=10, energy_every=1, **cfg["params"])
    s = Solver()
    s.load_workload(w)
    if case == "graph":
        W = gnn.init_weights(2).astype(np.float32)
        W[-2:] = [0.0, 0.6]
        s.gl_set_weights(W, np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.float32))
    s.set_params(**prm)
    X0 = _dev(wl.random_block(4, w.mesh.n_dofs, w.p))
    s.set_x0(X0, orthonormalize=True)
    ref, _, _ = s.step(cfg["steps"])
    xa = s.get_x().cpu().numpy()

    nb = s.workspace_size(w.p)
    ws = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s.set_workspace(ws)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    s.set_x0(X0, orthonormalize=True)
    got, _, _ = s.step(cfg["steps"])
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0, (free0, free1)
    assert len(got) == len(ref) == cfg["steps"]
    for x, y in zip(got, ref):
        for f in FIELDS:
            assert _same(x[f], y[f]), (case, f, x, y)
    assert np.array_equal(s.get_x().cpu().numpy(), xa)
    if case == "mixed":
        assert got[0]["precision"] == 1 and got[-1]["precision"] == 0   # the switch ran inside the workspace
    if case == "graph":
        assert 3 in [x["precond_used"] for x in got]

    # one piece short: a clean capacity error at set_x0 or in the first steps
    small = ws[: nb - 256]
    s.set_workspace(small)
    with pytest.raises(RuntimeError, match="workspace"):
        s.set_x0(X0, orthonormalize=True)
        s.step(cfg["steps"])
    # back to library allocation
    s.set_workspace(None)
    s.set_x0(X0, orthonormalize=True)
    again, _, _ = s.step(3)
    for x, y in zip(again, ref):
        assert _same(x["kkt"], y["kkt"])
    s.close()


@pytest.mark.parametrize("case", ["fp64", "mixed"])
def test_resume_into_a_workspace(case):
    """ofks_state_set on a context whose iteration state lives in a caller
    workspace: the resumed steps equal the uninterrupted run's bit for bit
    (FP64, and across the FP32 -> FP64 switch, whose FP64 set then comes from
    the region the workspace keeps for it)."""
    import torch
    from paper_2007_14228_amd import Solver
    cfg = dict(CASES[case])
    w = wl.make_workload("c1")
    print(f"[gpu] workspace resume {case}", flush=True)
    prm = dict(beta=w.beta, tol=1e-30, max_iter=500, pcg_iters=10, energy_every=1, **cfg["params"])
    k1, k2 = (5, 12) if case == "fp64" else (4, 50)
    a = Solver()
    a.load_workload(w)
    a.set_params(**prm)
    a.set_x0(_dev(wl.random_block(4, w.mesh.n_dofs, w.p)), orthonormalize=True)
    a.step(k1)
    state = a.state_get()
    ref, _, _ = a.step(k2)
    xa = a.get_x().cpu().numpy()
    b = Solver()
    b.load_workload(w)
    b.set_params(**prm)
    ws = torch.zeros(b.workspace_size(w.p), dtype=torch.uint8, device="cuda")
    b.set_workspace(ws)
    b.state_set(state)
    got, _, _ = b.step(k2)
    for x, y in zip(got, ref):
        for f in FIELDS:
            assert _same(x[f], y[f]), (case, f, x, y)
    assert np.array_equal(b.get_x().cpu().numpy(), xa)
    if case == "mixed":
        assert ref[0]["precision"] == 1 and ref[-1]["precision"] == 0
    a.close()
    b.close()
