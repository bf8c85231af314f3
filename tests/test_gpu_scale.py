"""The 96-nucleus cluster at full size (n ~ 8e6 interior DOFs, p = 512, the
precision form): n p > 2^31, so every block index is 64-bit here.

Checked against the oracle on sampled rows (fem.local_rows assembles just the
tetrahedra around them): the CSR pattern bit-exact, L, B, H to 1e-12; the
dual product (H X, B X) and the preconditioner's operator (L/2 - lam B) X in
FP64 (1e-12) and in FP32 (within 1e-5 of the row's absolute sum
sum_j |a_ij| |x_j|, a bound FP32 rounding of ~15-term sums meets with room);
then FP32 iterations run at this size.  The start block is drawn on the
device (workloads.device_random_block); the rows the checks need are copied
back.  About two minutes and up to ~200 GB of device memory."""
import time

import numpy as np
import pytest

import workloads as wl
from oracle import fem

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def c4():
    from paper_2007_14228_amd import Solver
    print("[gpu] c4: workload", flush=True)
    w = wl.make_workload("c4", seed=0)
    s = Solver()
    s.load_workload(w)
    print(f"[gpu] c4: n={w.mesh.n_dofs} nnz={s.nnz} p={w.p}; oracle rows", flush=True)
    rows = np.sort(np.random.default_rng(3).choice(w.mesh.n_dofs, 300, replace=False))
    loc = fem.local_rows(w.mesh, w.Z, w.R, rows)
    yield w, s, rows, loc
    s.close()


def test_c4_csr_on_sampled_rows(c4):
    w, s, rows, loc = c4
    assert w.mesh.n_dofs * w.p > 2 ** 31
    g = s.csr_get()
    for i in rows:
        cols, L, B, M = loc[int(i)]
        a, b = g["row_ptr"][i], g["row_ptr"][i + 1]
        assert np.array_equal(g["col"][a:b], cols)
        assert _relerr(g["L"][a:b], L) < 1e-12
        assert _relerr(g["B"][a:b], B) < 1e-12
        assert _relerr(g["H"][a:b], 0.5 * L + M) < 1e-12


def test_c4_products_on_sampled_rows(c4):
    """Both products in both precisions through the kernels the automatic
    choice takes at p = 512 (the LDS-halo SpMM: four 512-byte column slices
    per FP32 row, eight per FP64 row)."""
    import torch
    w, s, rows, loc = c4
    n, p = w.mesh.n_dofs, w.p
    print("[gpu] c4: X on the device", flush=True)
    X = wl.device_random_block(4, n, p)
    need = np.unique(np.concatenate([loc[int(i)][0] for i in rows]))
    Xneed = X.index_select(0, torch.from_numpy(need).to("cuda")).cpu().numpy()
    pos = {int(c): k for k, c in enumerate(need)}
    idx = torch.from_numpy(rows).to("cuda")
    lam = -np.linspace(0.05, 40.0, p)
    lam[[3, 200, 511]] = [0.0, 0.5, 2.0]            # identity-branch columns: zero output

    def oracle_rows(Xv):
        out = {}
        for j, i in enumerate(rows):
            cols, L, B, M = loc[int(i)]
            Xc = Xv[[pos[int(c)] for c in cols]]
            on = lam < 0
            shift = (0.5 * L) @ Xc - (B @ Xc) * lam
            shift[~on] = 0.0
            absb = dict(H=np.abs(0.5 * L + M) @ np.abs(Xc), B=np.abs(B) @ np.abs(Xc),
                        T=np.abs(0.5 * L) @ np.abs(Xc) + (np.abs(B) @ np.abs(Xc)) * np.abs(lam))
            out[j] = ((0.5 * L + M) @ Xc, B @ Xc, shift, absb)
        return out

    for prec in ("f64", "f32"):
        Xp = X if prec == "f64" else X.float()
        Xv = Xneed if prec == "f64" else Xneed.astype(np.float32).astype(np.float64)
        ref = oracle_rows(Xv)
        print(f"[gpu] c4: {prec} dual product", flush=True)
        HX, BX = s.spmm_ex(Xp, "dual")
        got = (HX.index_select(0, idx).double().cpu().numpy(), BX.index_select(0, idx).double().cpu().numpy())
        del HX, BX
        torch.cuda.empty_cache()
        print(f"[gpu] c4: {prec} shifted product", flush=True)
        Q = s.spmm_ex(Xp, "shift", lam)
        gotq = Q.index_select(0, idx).double().cpu().numpy()
        del Q
        torch.cuda.empty_cache()
        for j in range(len(rows)):
            rh, rb, rq, absb = ref[j]
            if prec == "f64":
                assert _relerr(got[0][j], rh) < 1e-12
                assert _relerr(got[1][j], rb) < 1e-12
                assert _relerr(gotq[j], rq) < 1e-12
            else:
                assert np.all(np.abs(got[0][j] - rh) <= 1e-5 * absb["H"])
                assert np.all(np.abs(got[1][j] - rb) <= 1e-5 * absb["B"])
                assert np.all(np.abs(gotq[j] - rq) <= 1e-5 * absb["T"])
            assert np.all(gotq[j][lam >= 0] == 0.0)
        if prec == "f32":
            del Xp
    del X
    torch.cuda.empty_cache()


def test_c4_fp32_iterations(c4):
    import torch
    w, s, rows, loc = c4
    n, p = w.mesh.n_dofs, w.p
    print("[gpu] c4: FP32 iterations", flush=True)
    X0 = wl.device_random_block(4, n, p)
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
                                      "pcg_sum", "bbdot")}
    print(f"[gpu] c4: {dt * 1e3:.1f} ms/iteration; " +
          " ".join(f"{k}={v[0] / max(v[1], 1):.3f}ms" for k, v in timers.items() if v[1]), flush=True)
    print("[gpu] c4: " + "; ".join(f"k={x['k']} kkt={x['kkt']:.4e} fea={x['fea']:.2e}" for x in st), flush=True)
    assert all(x["precision"] == 1 for x in st)
    assert all(np.isfinite(x["kkt"]) and np.isfinite(x["fea"]) for x in st)
    assert st[0]["fea"] < 1e-3                      # B-orthonormal start, in FP32
    assert st[-1]["kkt"] < st[0]["kkt"]
    # the FP64 refinement at this size: the switch converts the three state
    # blocks one at a time after freeing the FP32 scratch, so the FP64 set
    # (8 x 32.8 GB) fits beside the system
    free, total = torch.cuda.mem_get_info()
    print(f"[gpu] c4: device memory before the switch: {free / 2**30:.1f} GiB free of {total / 2**30:.1f}", flush=True)
    s.set_params(beta=w.beta, tol=1e-30, max_iter=7, precond="paper", pcg_iters=10, precision="f32",
                 refine_tol=1.0, energy_every=10)
    t = time.perf_counter()
    st2, _, _ = s.step(3)
    torch.cuda.synchronize()
    print(f"[gpu] c4: after the switch: " + "; ".join(f"k={x['k']} prec={x['precision']} kkt={x['kkt']:.4e}"
                                                     for x in st2) + f" ({time.perf_counter() - t:.1f} s)", flush=True)
    assert st2[0]["precision"] == 1 and st2[-1]["precision"] == 0
    assert all(np.isfinite(x["kkt"]) and np.isfinite(x["fea"]) for x in st2)
