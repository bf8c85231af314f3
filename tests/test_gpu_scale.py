"""The 96-nucleus cluster at full size (n ~ 8e6 interior DOFs, p = 512, the
precision form): n p > 2^31, so every block index is 64-bit here.

Opt-in (it takes minutes and ~200 GB of device memory): OFKS_SCALE=1.
Checked against the oracle on sampled rows (fem.local_rows assembles just the
tetrahedra around them): the CSR pattern bit-exact, L, B, H and the FP64 dual
SpMM to 1e-12; then FP32 iterations run at this size (the FP64 refinement
does not fit next to the FP32 blocks on one GPU)."""
import os
import time

import numpy as np
import pytest

import workloads as wl
from oracle import fem

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("OFKS_SCALE") != "1",
                                 reason="full-size 96-nucleus run: set OFKS_SCALE=1")]


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_c4_full_size():
    import torch
    from paper_2007_14228_amd import Solver
    print("[gpu] c4: workload", flush=True)
    w = wl.make_workload("c4", seed=0)
    n, p = w.mesh.n_dofs, w.p
    assert n * p > 2 ** 31
    s = Solver()
    s.load_workload(w)
    print(f"[gpu] c4: n={n} nnz={s.nnz} p={p}; CSR on sampled rows", flush=True)
    rows = np.sort(np.random.default_rng(3).choice(n, 300, replace=False))
    loc = fem.local_rows(w.mesh, w.Z, w.R, rows)
    g = s.csr_get()
    for i in rows:
        cols, L, B, M = loc[int(i)]
        a, b = g["row_ptr"][i], g["row_ptr"][i + 1]
        assert np.array_equal(g["col"][a:b], cols)
        assert _relerr(g["L"][a:b], L) < 1e-12
        assert _relerr(g["B"][a:b], B) < 1e-12
        assert _relerr(g["H"][a:b], 0.5 * L + M) < 1e-12
    del g
    print("[gpu] c4: X0 (FP64, streamed) and the dual SpMM on sampled rows", flush=True)
    need = np.unique(np.concatenate([loc[int(i)][0] for i in rows]))
    Xneed = np.empty((len(need), p))
    X0 = torch.empty((n, p), dtype=torch.float64, device="cuda")
    for r0, r1, chunk in wl.random_block_chunks(4, n, p):
        X0[r0:r1].copy_(torch.from_numpy(chunk))
        m = (need >= r0) & (need < r1)
        Xneed[m] = chunk[need[m] - r0]
    HX, BX = s.spmm(X0)
    idx = torch.from_numpy(rows).to("cuda")
    HXs = HX.index_select(0, idx).cpu().numpy()
    BXs = BX.index_select(0, idx).cpu().numpy()
    del HX, BX
    torch.cuda.empty_cache()
    pos = {int(c): k for k, c in enumerate(need)}
    for j, i in enumerate(rows):
        cols, L, B, M = loc[int(i)]
        Xc = Xneed[[pos[int(c)] for c in cols]]
        assert _relerr(HXs[j], (0.5 * L + M) @ Xc) < 1e-12
        assert _relerr(BXs[j], B @ Xc) < 1e-12
    print("[gpu] c4: FP32 iterations", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=4, precond="paper", pcg_iters=10, precision="f32",
                 refine_tol=0.0, energy_every=10)
    s.set_x0(X0, orthonormalize=True)
    del X0
    torch.cuda.empty_cache()
    s.timing(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st, _, _ = s.step(4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / len(st)
    timers = {k: s.timer(k) for k in ("spmm_dual", "spmm_shift", "gram", "update_a", "update_b", "pcg_r", "pcg_dx",
                                      "bbdot")}
    print(f"[gpu] c4: {dt * 1e3:.1f} ms/iteration; " +
          " ".join(f"{k}={v[0] / max(v[1], 1):.3f}ms" for k, v in timers.items() if v[1]), flush=True)
    print("[gpu] c4: " + "; ".join(f"k={x['k']} kkt={x['kkt']:.4e} fea={x['fea']:.2e}" for x in st), flush=True)
    assert all(x["precision"] == 1 for x in st)
    assert all(np.isfinite(x["kkt"]) and np.isfinite(x["fea"]) for x in st)
    assert st[0]["fea"] < 1e-3                      # B-orthonormal start, in FP32
    assert st[-1]["kkt"] < st[0]["kkt"]
    # the same iteration continued through each SpMM kernel (FP32, four 512-byte slices per row), timed
    for mode in ("gather", "halo"):
        s.set_params(beta=w.beta, tol=1e-30, max_iter=100, precond="paper", pcg_iters=10, precision="f32",
                     refine_tol=0.0, energy_every=10, spmm_mode=mode)
        s.timing(True)
        st2, _, _ = s.step(2)
        ms, cnt = s.timer("spmm_shift")
        md, cd = s.timer("spmm_dual")
        print(f"[gpu] c4: spmm {mode}: shift {ms / max(cnt, 1):.3f} ms x {cnt}, dual {md / max(cd, 1):.3f} ms; "
              f"kkt={st2[-1]['kkt']:.4e}", flush=True)
        assert all(np.isfinite(x["kkt"]) for x in st2)
