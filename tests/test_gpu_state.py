"""Checkpoint/resume and the density update, through the C ABI.

ofks_state_get at step k, then ofks_state_set on a fresh context with the
same system and parameters: the following steps must reproduce the
uninterrupted run bit for bit (every reduction has a fixed order), in FP64,
across the FP32 -> FP64 switch of the precision form, in the SCF iteration
(the Hartree potential that warm-starts the next solve is part of the state)
and in the graph learned form (its fallback state is part of the state).

ofks_update_density: H(X) re-assembled from the iterate's density against
the oracle's H(X) (1e-10 relative)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import fem, gnn, pcal, scf

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
    Z = np.array([3.0, 1.0])
    R = np.array([[-1.2, 0.0, 0.0], [1.2, 0.0, 0.0]])
    return wl.Workload("lih", mesh, Z, R, p=2, beta=1.0, scf=True, seed=0)


CASES = {
    "fp64": dict(wk="c1", params=dict(precond="paper"), k1=9, k2=12),
    "mixed": dict(wk="c1", params=dict(precond="paper", precision="f32", refine_tol=0.1), k1=4, k2=50),
    "scf": dict(wk="lih", params=dict(precond="paper", scf=1), k1=7, k2=8),
    "graph": dict(wk="c1", params=dict(precond="graph", fallback_stall=6), k1=10, k2=30),
}


@pytest.mark.parametrize("case", list(CASES))
def test_resume_is_bit_identical(case):
    from paper_2007_14228_amd import Solver
    cfg = CASES[case]
    w = wl.make_workload("c1") if cfg["wk"] == "c1" else _lih()
    print(f"[gpu] resume {case}", flush=True)
    prm = dict(beta=w.beta, tol=1e-30, max_iter=500, pcg_iters=10, energy_every=1, **cfg["params"])
    W = gnn.init_weights(2).astype(np.float32)
    W[-2:] = [0.0, 0.6]
    norm = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.float32)

    def fresh():
        s = Solver()
        s.load_workload(w)
        if case == "graph":
            s.gl_set_weights(W, norm)
        s.set_params(**prm)
        return s

    a = fresh()
    a.set_x0(_dev(wl.random_block(4, w.mesh.n_dofs, w.p)), orthonormalize=True)
    first, _, _ = a.step(cfg["k1"])
    state = a.state_get()
    ref, _, _ = a.step(cfg["k2"])
    xa = a.get_x().cpu().numpy()
    b = fresh()
    b.set_x0(_dev(wl.random_block(9, w.mesh.n_dofs, w.p)), orthonormalize=True)   # replaced by the state
    b.state_set(state)
    got, _, _ = b.step(cfg["k2"])
    assert len(got) == len(ref) == cfg["k2"]
    for x, y in zip(got, ref):
        for f in FIELDS:
            assert _same(x[f], y[f]), (case, f, x, y)
    assert np.array_equal(b.get_x().cpu().numpy(), xa)
    if case == "mixed":
        assert ref[0]["precision"] == 1 and ref[-1]["precision"] == 0   # the switch happened after the checkpoint
    if case == "graph":
        kinds = [x["precond_used"] for x in first + ref]
        assert 1 in kinds and 3 in kinds                                  # the fallback state was exercised
    a.close()
    b.close()


def test_state_set_rejects_a_foreign_buffer():
    import torch
    from paper_2007_14228_amd import Solver
    w = wl.make_workload("c1")
    s = Solver()
    s.load_workload(w)
    s.set_params(beta=w.beta, precond="paper")
    junk = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        s.state_set(junk)
    s.close()


def test_update_density_builds_the_hamiltonian_of_the_iterate():
    from paper_2007_14228_amd import Solver
    w = _lih()
    d = fem.discretize(w.mesh, w.Z, w.R)
    print("[gpu] update_density", flush=True)
    prob = scf.KSProblem(d, w.Z, w.R)
    X = pcal.chol_gs(prob, wl.random_block(13, d.n, w.p))
    Href, _, _, _ = prob.build(X)
    s = Solver()
    s.load_workload(w)
    s.set_params(beta=w.beta, precond="paper", scf=1)
    s.set_x0(_dev(X), orthonormalize=False)
    s.update_density()
    H = s.csr_get()["H"]
    assert float(np.abs(H - Href).max() / np.abs(Href).max()) < 1e-10
    s.close()
