"""Training pipeline of the learned pointwise preconditioner.

1. Collect samples: run the plain method (FP64, the paper preconditioner) on
   seeded training workloads; while it iterates, the library records
   (features, a, t, w) for every `row_stride`-th row and all columns
   (ofks_lp_collect): by default the energy-norm objective, which fits the
   scale s node by node to minimize the quadratic model of T over s J g.
2. Train: full-batch Adam on the device (ofks_lp_train), hand-written forward
   and backward kernels.
3. Save the 193 weights and the 8 standardization constants as JSON.

    python -m paper_2007_14228_amd.learned --seeds 1000:1200 --out weights.json

Workloads, samples and training all run on the GPU through the library; this
module only sequences the calls.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "lp_weights.json")


def init_weights(seed: int) -> np.ndarray:
    """Small random first layer, zero output layer: the untrained network is
    the Jacobi preconditioner of the paper's operator."""
    rng = np.random.default_rng(seed)
    W = np.zeros(193, dtype=np.float32)
    W[:128] = rng.standard_normal(128) * 0.5
    W[128:160] = rng.standard_normal(32) * 0.1
    return W


def collect(seeds, kind: str = "c2", target_dofs: int = 200_000, iters: int = 60, row_stride: int = 64,
            cap: int = 40_000_000, pcg_iters: int = 10, objective: str = "energy", log=print):
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as wl
    from . import Solver
    buf = torch.zeros((cap, 8), dtype=torch.float32, device="cuda")
    count = 0
    for seed in seeds:
        t = time.perf_counter()
        w = wl.make_workload(kind, seed=seed, target_dofs=target_dofs)
        s = Solver()
        s.load_workload(w)
        s.set_params(beta=w.beta, tol=1e-30, max_iter=iters, precond="paper", pcg_iters=pcg_iters,
                     scf=1 if w.scf else 0, energy_every=10)
        X0 = torch.from_numpy(wl.random_block(seed, w.mesh.n_dofs, w.p)).cuda()
        s.set_x0(X0, orthonormalize=True)
        view = buf[count:]
        if view.shape[0] == 0:
            break
        s.lp_collect(view, row_stride, objective)
        s.step(iters + 1)
        got = s.lp_collected()
        s.lp_collect(None, 0)
        s.close()
        count += got
        log(f"[learned] seed {seed}: n={w.mesh.n_dofs} p={w.p} samples={got} total={count} "
            f"({time.perf_counter() - t:.1f}s)")
    return buf[:count]


def train(samples, epochs: int = 2000, lr: float = 3e-3, seed: int = 0):
    from . import Solver
    s = Solver()
    W, norm, losses = s.lp_train(samples, epochs, lr, init_weights(seed))
    s.close()
    return W, norm, losses


DEFAULT_GRAPH_WEIGHTS = os.path.join(HERE, "gl_weights.json")


def init_graph_weights(seed: int, ft: float = 0.5) -> np.ndarray:
    """Graph form: small random first layer, zero output weights and output
    biases (0, ft): the untrained network is one Jacobi sweep through T after
    the Jacobi scaling, damped by ft."""
    rng = np.random.default_rng(seed)
    W = np.zeros(226, dtype=np.float32)
    W[:128] = rng.standard_normal(128) * 0.5
    W[128:160] = rng.standard_normal(32) * 0.1
    W[-2:] = [0.0, ft]
    return W


def train_graph(seeds, kind: str = "c2", target_dofs: int = 200_000, iters: int = 60, every: int = 5,
                slots: int = 12, epochs: int = 3, lr: float = 2e-3, pcg_iters: int = 10, log=print):
    """The graph form, trained on gradient blocks of the plain method (FP64,
    paper preconditioner, fixed H = L/2 + M_ext of each seeded workload): for
    each seed, the library captures G and the shifts of every `every`-th
    iterate, then takes `epochs` passes of Adam over them on that system; the
    weights and the optimizer state carry over to the next seed.  The feature
    standardization comes from the first workload."""
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as wl
    from . import Solver
    W = init_graph_weights(0)
    adam = np.zeros(453, dtype=np.float32)
    norm = None
    history = []
    for seed in seeds:
        t = time.perf_counter()
        w = wl.make_workload(kind, seed=seed, target_dofs=target_dofs)
        s = Solver()
        s.load_workload(w)
        n, p = w.mesh.n_dofs, w.p
        if norm is None:
            norm = s.gl_feature_norm()
        buf = torch.zeros((slots, n, p), dtype=torch.float64, device="cuda")
        s.set_params(beta=w.beta, tol=1e-30, max_iter=iters, precond="paper", pcg_iters=pcg_iters, scf=0,
                     energy_every=10)
        s.gl_capture(buf, every=every)
        s.set_x0(torch.from_numpy(wl.random_block(seed, n, p)).cuda(), orthonormalize=True)
        s.step(iters + 1)
        count, lam = s.gl_captured(p)
        s.gl_capture(None)
        if count == 0:
            s.close()
            continue
        s.gl_set_weights(W, norm)
        W, adam, losses = s.gl_train(buf[:count], lam, epochs, lr, W, adam)
        s.close()
        history.append(dict(seed=seed, blocks=count, loss_first=float(losses[0].mean()),
                            loss_last=float(losses[-1].mean())))
        log(f"[learned] graph seed {seed}: n={n} p={p} blocks={count} loss {losses[0].mean():.5f} -> "
            f"{losses[-1].mean():.5f} ({time.perf_counter() - t:.1f}s)")
    return W, norm, history


def save(path: str, W, norm, meta: dict):
    with open(path, "w") as f:
        json.dump(dict(weights=[float(x) for x in W], norm=[float(x) for x in norm], meta=meta), f, indent=1)


def load(path: str = DEFAULT_WEIGHTS):
    d = json.load(open(path))
    return np.asarray(d["weights"], dtype=np.float32), np.asarray(d["norm"], dtype=np.float32), d.get("meta", {})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--form", default="pointwise", choices=["pointwise", "graph"])
    ap.add_argument("--every", type=int, default=5, help="graph form: capture every k-th iterate")
    ap.add_argument("--slots", type=int, default=12, help="graph form: blocks captured per workload")
    ap.add_argument("--seeds", default="1000:1200")
    ap.add_argument("--kind", default="c2")
    ap.add_argument("--target-dofs", type=int, default=200_000)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--row-stride", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--objective", default="energy", choices=["energy", "euclid"])
    ap.add_argument("--cap", type=float, default=4e7, help="sample capacity")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args()
    lo, hi = (int(x) for x in a.seeds.split(":"))
    if a.form == "graph":
        t = time.perf_counter()
        W, norm, hist = train_graph(range(lo, hi), a.kind, a.target_dofs, a.iters, a.every, a.slots, a.epochs, a.lr)
        out = a.out if a.out != DEFAULT_WEIGHTS else DEFAULT_GRAPH_WEIGHTS
        meta = dict(form="graph", seeds=a.seeds, kind=a.kind, h="fixed L/2 + M_ext", target_dofs=a.target_dofs,
                    iters=a.iters, every=a.every, slots=a.slots, epochs=a.epochs, lr=a.lr,
                    blocks=int(sum(h["blocks"] for h in hist)), loss_first=hist[0]["loss_first"] if hist else None,
                    loss_last=hist[-1]["loss_last"] if hist else None, seconds=time.perf_counter() - t)
        save(out, W, norm, meta)
        print(json.dumps(meta))
        return
    t = time.perf_counter()
    S = collect(range(lo, hi), a.kind, a.target_dofs, a.iters, a.row_stride, int(a.cap), objective=a.objective)
    t_collect = time.perf_counter() - t
    t = time.perf_counter()
    W, norm, losses = train(S, a.epochs, a.lr)
    t_train = time.perf_counter() - t
    meta = dict(seeds=a.seeds, kind=a.kind, objective=a.objective, target_dofs=a.target_dofs, iters=a.iters,
                row_stride=a.row_stride,
                samples=int(S.shape[0]), epochs=a.epochs, lr=a.lr, loss_first=float(losses[0]),
                loss_last=float(losses[-1]), seconds_collect=t_collect, seconds_train=t_train)
    save(a.out, W, norm, meta)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
