#!/usr/bin/env python3
"""Benchmark of the PCAL hot path on one MI355X.

Workload (default "c3"): a seeded 24-nucleus cluster (Z in {1,6,7,8}) on a
graded P1 tetrahedral mesh with n ~ 2e6 interior DOFs and p = 128 orbitals,
fixed Hamiltonian H = L/2 + M_ext.  One step = one PCAL iteration: dual SpMM,
Gram, multiplier, gradient/kkt, the paper's preconditioner (Jacobi-PCG,
m = 10 inner iterations), BB2 step and update, all in FP64.

Printed (one JSON line): iterations per second over exactly --steps timed
iterations after --warmup untimed ones, the roofline of the dominant kernel
(the preconditioner's shifted SpMM) from HIP-event kernel timings, the time to
residual 1e-6 for the plain FP64 method and for the mixed-precision form, and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to residual 1e-6 + iter/s: FP64 plain vs mixed-prec + learned precond"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "u2", "u3"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--pcg-iters", type=int, default=10)
    ap.add_argument("--no-converge", action="store_true", help="skip the time-to-residual runs")
    ap.add_argument("--cpu-baseline", default="auto", choices=["auto", "skip"])
    ap.add_argument("--max-iter", type=int, default=1500)
    ap.add_argument("--poisson-adapt", type=float, default=0.0,
                    help="SCF workloads: Hartree CG tolerance max(1e-12, this x the previous residual) (0: 1e-12)")
    ap.add_argument("--energy-legs", default="both", choices=["both", "fp64", "mixed"],
                    help="which runs --energy-check makes (one per process for the largest workloads)")
    ap.add_argument("--energy-check", type=float, default=0.0,
                    help="also run FP64 and mixed precision to this residual and report the energy difference")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (known bytes) for HBM counter calibration")
    ap.add_argument("--study-steps", default=None, metavar="A:B",
                    help="also run FP64 to residual 1e-6 for workload seeds A..B-1 under each step rule (BB2, BB1, "
                         "ABB1, ABB2) with the paper preconditioner, and BB2 without one; report iterations")
    ap.add_argument("--study-p", default=None, metavar="P1,P2,...",
                    help="also time FP64 iterations of the same workload at these block widths and report each "
                         "kernel's share of an iteration, and the host's p x p share")
    ap.add_argument("--study-m", default=None, metavar="M1,M2,...",
                    help="also run FP64 to residual 1e-6 with the paper preconditioner at these inner PCG lengths m")
    ap.add_argument("--study-c5", default=None, metavar="A:B",
                    help="held-out evaluation: for workload seeds A..B-1, time to residual 1e-6 of the plain FP64 "
                         "method and the mixed-precision forms with the paper, learned and graph preconditioners")
    ap.add_argument("--jsonl", default=None, metavar="PATH",
                    help="after the timed steps, run --steps more one at a time and write one JSON line per "
                         "iteration (residuals, energy, step, wall ms and each kernel class's ms)")
    return ap.parse_args()


P_STUDY_TIMERS = ("spmm_dual", "spmm_shift", "gram", "update_a", "update_b", "pcg_r", "pcg_dx", "pcg_sum", "bbdot",
                  "density", "poisson", "assemble_h", "mlp", "graph", "host")


def p_study(torch, a, s, w, params, steps=3, warmup=2):
    """Per-kernel share of an FP64 iteration against the block width p at a
    fixed mesh (the single-GPU analogue of the paper's per-part cost figure)."""
    import workloads as wl
    n = w.mesh.n_dofs
    rows = []
    for p in (int(v) for v in a.study_p.split(",")):
        X0 = torch.from_numpy(wl.random_block(2000 + p, n, p)).to("cuda")
        s.set_params(tol=1e-30, **dict(params, max_iter=warmup + steps + 5, energy_every=10 if p > 64 else 1))
        s.set_x0(X0, orthonormalize=True)
        del X0
        s.step(warmup)
        s.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _, _ = s.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / len(st)
        ms = {k: s.timer(k)[0] / len(st) for k in P_STUDY_TIMERS}
        s.timing(False)
        ms = {k: round(v, 3) for k, v in ms.items() if v > 0}
        share = {k: round(v / (dt * 1e3), 3) for k, v in ms.items()}
        log(f"  p={p}: {dt * 1e3:.1f} ms/iteration; " + " ".join(f"{k}={v:.0%}" for k, v in share.items()))
        rows.append(dict(p=p, ms_per_iteration=round(dt * 1e3, 3), kernel_ms=ms, share=share))
    return dict(workload=a.workload, n=n, precision="f64", precond=params["precond"], pcg_iters=params["pcg_iters"],
                note="host = the serial p x p algebra on the host (the paper's non-parallel part); every other "
                     "entry is a device kernel class", rows=rows)


def step_rule_study(torch, a, params):
    """Section 4.4's comparison of the BB step rules (and Section 5's check
    that the preconditioner helps) on seeded workloads of one kind: FP64, same
    X0 per seed, residual 1e-6, iterations and seconds per (rule, preconditioner)."""
    import workloads as wl
    from paper_2007_14228_amd import Solver
    lo, hi = (int(v) for v in a.study_steps.split(":"))
    cases = [("bb2", "paper"), ("bb1", "paper"), ("abb1", "paper"), ("abb2", "paper"), ("bb2", "none")]
    runs = []
    for seed in range(lo, hi):
        w = wl.make_workload(a.workload, seed=seed)
        X0 = torch.from_numpy(wl.random_block(1000 + seed, w.mesh.n_dofs, w.p)).to("cuda")
        s = Solver()
        s.load_workload(w)
        for rule, pre in cases:
            r = run_to_tol(torch, s, X0, 1e-6, dict(params, beta=w.beta, scf=1 if w.scf else 0, step_rule=rule,
                                                    precond=pre))
            log(f"  seed {seed} {rule}/{pre}: {r['iterations']} iterations, {r['seconds']} s, rel {r['rel']:.2e}")
            runs.append(dict(seed=seed, step_rule=rule, precond=pre, iterations=r["iterations"],
                             seconds=r["seconds"], converged=r["converged"], rel=r["rel"], energy=r["energy"]))
        s.close()
    summary = {}
    for rule, pre in cases:
        rs = [r for r in runs if r["step_rule"] == rule and r["precond"] == pre]
        conv = [r for r in rs if r["converged"]]
        summary[f"{rule}/{pre}"] = dict(
            converged=f"{len(conv)}/{len(rs)}",
            median_iterations=float(np.median([r["iterations"] for r in conv])) if conv else None,
            mean_seconds=round(float(np.mean([r["seconds"] for r in conv])), 3) if conv else None)
    return dict(workload=a.workload, seeds=f"{lo}:{hi}", tol=1e-6, max_iter=params["max_iter"], runs=runs,
                summary=summary)


def m_study(torch, a, s, X0, params):
    """The paper preconditioner's inner-solve length: the paper fixes no m
    (eq. precondition-T); FP64 time to residual 1e-6 at each m."""
    rows = []
    for m in (int(v) for v in a.study_m.split(",")):
        r = run_to_tol(torch, s, X0, 1e-6, dict(params, pcg_iters=m))
        log(f"  m={m}: {r['iterations']} iterations, {r['seconds']} s, rel {r['rel']:.2e}")
        rows.append(dict(m=m, iterations=r["iterations"], seconds=r["seconds"], converged=r["converged"],
                         iter_per_s=r["iter_per_s"], energy=r["energy"]))
    return dict(workload=a.workload, precision="f64", tol=1e-6, rows=rows)


def graph_untrained():
    """The graph form with untrained heads: output weights 0, biases (0, 0.65),
    i.e. one Jacobi sweep through T damped by 0.65 after the Jacobi scaling."""
    from paper_2007_14228_amd import learned
    return learned.init_graph_weights(0, 0.65), np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.float32)


def learned_legs(torch, s, X0, mparams):
    """The mixed-precision forms with the learned preconditioners (energy and
    stall fallbacks on), each from the same start."""
    from paper_2007_14228_amd import learned
    legs = {}
    wpath = learned.DEFAULT_WEIGHTS
    if os.path.exists(wpath):
        Wl, norml, meta = learned.load(wpath)
        log(f"time to residual 1e-6: mixed precision + learned pointwise preconditioner ({os.path.basename(wpath)})")
        s.lp_set_weights(Wl, norml)
        legs["mixed_learned_precond"] = run_to_tol(torch, s, X0, 1e-6, dict(mparams, precond="learned",
                                                                              energy_every=1))
        legs["mixed_learned_precond"]["weights"] = {"file": os.path.relpath(wpath, ROOT),
                                                    **{k: meta[k] for k in ("seeds", "kind", "samples") if k in meta}}
        log(f"  {legs['mixed_learned_precond']}")
    log("time to residual 1e-6: mixed precision + learned pointwise form, untrained network (Jacobi of T)")
    s.lp_set_weights(learned.init_weights(0), np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.float32))
    legs["mixed_learned_form_untrained"] = run_to_tol(torch, s, X0, 1e-6, dict(mparams, precond="learned",
                                                                               energy_every=1))
    log(f"  {legs['mixed_learned_form_untrained']}")
    log("time to residual 1e-6: mixed precision + graph form, untrained heads (damped sweep through T)")
    s.gl_set_weights(*graph_untrained())
    legs["mixed_graph_form_untrained"] = run_to_tol(torch, s, X0, 1e-6, dict(mparams, precond="graph",
                                                                             energy_every=1))
    log(f"  {legs['mixed_graph_form_untrained']}")
    log("time to residual 1e-6: mixed precision + graph form, fixed heads, five sweeps, no fallback")
    legs["mixed_graph_5_sweeps_alone"] = run_to_tol(torch, s, X0, 1e-6, dict(mparams, precond="graph", energy_every=1,
                                                                             graph_sweeps=5, fallback_window=0,
                                                                             fallback_stall=0))
    log(f"  {legs['mixed_graph_5_sweeps_alone']}")
    return legs


def c5_study(torch, a, params):
    """Held-out evaluation on workloads of the benchmark's kind: per seed, the
    same start for every leg; medians over the seeds that converged."""
    import workloads as wl
    from paper_2007_14228_amd import Solver
    lo, hi = (int(v) for v in a.study_c5.split(":"))
    runs = []
    for seed in range(lo, hi):
        t = time.perf_counter()
        w = wl.make_workload(a.workload, seed=seed)
        X0 = torch.from_numpy(wl.random_block(1000 + seed, w.mesh.n_dofs, w.p)).to("cuda")
        s = Solver()
        s.load_workload(w)
        prm = dict(params, beta=w.beta)
        legs = {"fp64_paper_precond": run_to_tol(torch, s, X0, 1e-6, prm)}
        mprm = dict(prm, precision="f32", refine_tol=1.5e-6)
        legs["mixed_paper_precond"] = run_to_tol(torch, s, X0, 1e-6, mprm)
        legs.update(learned_legs(torch, s, X0, mprm))
        s.close()
        del X0
        torch.cuda.empty_cache()
        for k, v in legs.items():
            runs.append(dict(seed=seed, leg=k, seconds=v["seconds"], iterations=v["iterations"],
                             converged=v["converged"], fallbacks=v["fallbacks"], energy=v["energy"]))
        log(f"  c5 seed {seed} ({time.perf_counter() - t:.0f} s): " +
            ", ".join(f"{k} {v['seconds']} s/{v['iterations']}it{'' if v['converged'] else ' (not converged)'}"
                      for k, v in legs.items()))
    summary = {}
    for leg in dict.fromkeys(r["leg"] for r in runs):
        rs = [r for r in runs if r["leg"] == leg]
        conv = [r for r in rs if r["converged"]]
        summary[leg] = dict(converged=f"{len(conv)}/{len(rs)}",
                            median_seconds=float(np.median([r["seconds"] for r in conv])) if conv else None,
                            median_iterations=float(np.median([r["iterations"] for r in conv])) if conv else None)
    return dict(workload=a.workload, seeds=f"{lo}:{hi}", tol=1e-6, runs=runs, summary=summary)


def jsonl_log(torch, s, steps, path):
    """One JSON line per iteration: the iterate's residuals, energy and step,
    the iteration's wall time and each kernel class's time (HIP events)."""
    names = P_STUDY_TIMERS + ("mlp_train", "graph_train")
    with open(path, "w") as f:
        for _ in range(steps):
            s.timing(True)
            st, done, _ = s.step(1)
            if not st:
                break
            x = st[0]
            ks = {k: round(s.timer(k)[0], 4) for k in names if s.timer(k)[1]}
            s.timing(False)
            f.write(json.dumps(dict(k=x["k"], kkt=x["kkt"], fea=x["fea"], rel=x["rel"], energy=x["energy"],
                                    eta=x["eta"], precond=x["precond_used"], precision=x["precision"],
                                    ms=round(x["ms"], 4), kernel_ms=ks)) + "\n")
            if done:
                break


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_spmm_shift(n, nnz, p, w):
    """One launch of the preconditioner operator Q = (L/2 - lam B) D: read D
    once, write Q once, read the CSR (values of L/2 and B, column index) and
    the row pointers."""
    return n * p * w * 2 + nnz * (2 * w + 4) + 8 * (n + 1)


def algorithmic_bytes_spmm_dual(n, nnz, p, w):
    return n * p * w * 3 + nnz * (2 * w + 4) + 8 * (n + 1)


def traffic_from_profiles(kernel, workload):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs,
    valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}@{workload}")
    except Exception:
        return None
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2007_14228_amd", "csrc", rec.get("source", "k_spmm.hip"))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if h != rec.get("source_sha"):
        return None
    return dict(bytes=rec.get("bytes_per_launch"), commit=rec.get("commit"), command=rec.get("command"),
                fetch_scale=rec.get("fetch_scale"), write_scale=rec.get("write_scale"))


def set_start(torch, s, X0):
    """set_x0 from a device block, or from a callable that makes one; then
    the previous run's blocks are released before the block is made, and the
    block is released before the first step (the library allocates the rest
    of its FP64 blocks then), which the largest workloads need."""
    if callable(X0):
        s.set_workspace(None)   # releases the previous run's blocks first
        torch.cuda.synchronize()
        X = X0()
        s.set_x0(X, orthonormalize=True)
        del X
        torch.cuda.empty_cache()
    else:
        s.set_x0(X0, orthonormalize=True)
    torch.cuda.synchronize()


def run_to_tol(torch, s, X0, tol, params, weights=None, chunk=100):
    """Seconds from the first step to the first iterate with residual < tol
    (setup excluded; X0 B-orthonormalized before the clock starts).  The
    steps are taken `chunk` at a time (the iteration state carries over), with
    a progress line after each chunk once a run has taken 20 s."""
    s.set_params(tol=tol, **params)
    if weights is not None:
        s.lp_set_weights(*weights)
    set_start(torch, s, X0)
    t0 = time.perf_counter()
    stats = []
    left = params.get("max_iter", 1000) + 1
    while left > 0:
        st, done, rc = s.step(min(chunk, left))
        stats += st
        left -= len(st)
        if done or not st:
            break
        if time.perf_counter() - t0 > 20.0:
            log(f"    {len(stats)} iterations, rel {st[-1]['rel']:.3e} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    last = stats[-1]
    iters = len(stats) - 1
    kinds = [0, 0, 0, 0]
    for x in stats[:-1]:
        kinds[x["precond_used"]] += 1
    return dict(seconds=round(dt, 3), iterations=iters, rel=last["rel"], energy=float(s.energy()[4]),
                converged=bool(last["rel"] < tol), iter_per_s=round(iters / dt, 3) if dt > 0 else None,
                iterations_by_precond={"none": kinds[0], "paper": kinds[1], "learned": kinds[2], "graph": kinds[3]},
                fallbacks=int(sum(x["fell_back"] for x in stats)),
                fp32_iterations=int(sum(1 for x in stats[:-1] if x["precision"] == 1)))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, X0_host, pcg_iters, iters=2):
    """The oracle as it stands, timed over `iters` PCAL iterations with the
    paper preconditioner on the full workload, reported as iterations per
    second.  From a random start every Lambda_ll is positive at k = 0, so
    iteration 0 takes the identity branch (no inner solve); the clock
    therefore runs from the evaluation of X^1 to that of X^(1+iters), i.e.
    over steady-state iterations that include the inner solves."""
    from oracle import fem, pcal, scf
    log("cpu baseline: oracle discretization")
    t = time.perf_counter()
    d = fem.discretize(w.mesh, w.Z, w.R)
    setup = time.perf_counter() - t
    if w.scf:
        prob = scf.KSProblem(d, w.Z, w.R)       # H(X) rebuilt every iteration
    else:
        prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, X0_host)
    log(f"cpu baseline: setup {setup:.1f}s; timing iterations 1..{iters}")
    stamps = {}

    def at_iterate(k, *_):                      # called once X^k is evaluated (HX, BX, Gram)
        stamps[k] = time.perf_counter()

    t = time.perf_counter()
    pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-30, max_iter=1 + iters, precond="paper",
                                    pcg_iters=pcg_iters), callback=at_iterate)
    total = time.perf_counter() - t
    dt = stamps[1 + iters] - stamps[1]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=iters / dt, unit="iter/s", cores=threads, kind="oracle",
                cpu=cpu_model(), host_cpus=os.cpu_count(),
                sample=f"PCAL iterations 1..{iters} (each with the m={pcg_iters} inner solves of the paper "
                       f"preconditioner) of the same workload from the same start, FP64, timed from the "
                       f"evaluation of X^1 to that of X^{1 + iters}: {dt:.2f} s; iteration 0 (identity branch) and "
                       f"the oracle setup ({setup:.1f} s) are not included; {total:.1f} s in all")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "design only)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(2)
    import workloads as wl
    from paper_2007_14228_amd import Solver

    t = time.perf_counter()
    w = wl.make_workload(a.workload, seed=a.seed, **({"progress": log} if a.workload.startswith("u") else {}))
    n = w.mesh.n_dofs
    p = w.p
    log(f"workload {a.workload}: n={n} p={p} tets={w.mesh.n_tets} ({time.perf_counter() - t:.1f}s)")
    X0_host = wl.random_block(1000 + a.seed, n, p)

    def X0():
        return torch.from_numpy(X0_host).to("cuda")

    s = Solver()
    t = time.perf_counter()
    s.load_workload(w)
    torch.cuda.synchronize()
    log(f"device assembly {time.perf_counter() - t:.2f}s nnz={s.nnz}")
    params = dict(beta=w.beta, precond="paper", pcg_iters=a.pcg_iters, max_iter=a.max_iter,
                  scf=1 if w.scf else 0, energy_every=10 if p > 64 else 1, poisson_adapt=a.poisson_adapt)
    s.set_params(tol=1e-30, **params)
    set_start(torch, s, X0)
    s.step(a.warmup)
    s.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, _, _ = s.step(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if len(stats) != a.steps:
        raise RuntimeError("fewer steps than requested")
    timers = {k: s.timer(k) for k in P_STUDY_TIMERS}
    s.timing(False)
    log(f"{a.steps} steps in {dt:.3f}s; rel={stats[-1]['rel']:.3e}")
    for k, (ms, cnt) in timers.items():
        if cnt:
            log(f"  {k:11s} {ms / cnt:8.3f} ms x {cnt}")

    nnz = s.nnz
    wbytes = 8
    ms_shift, cnt_shift = timers["spmm_shift"]
    if cnt_shift:
        avg = ms_shift / cnt_shift
        alg = algorithmic_bytes_spmm_shift(n, nnz, p, wbytes)
        kern = "k_spmm_shift"
    else:
        ms_d, cnt_d = timers["spmm_dual"]
        avg = ms_d / cnt_d
        alg = algorithmic_bytes_spmm_dual(n, nnz, p, wbytes)
        kern = "k_spmm_pair"
    achieved = alg / (avg * 1e-3) / 1e9
    # traffic: HBM bytes per launch from the committed rocprofv3 counter runs
    # (not measured in this run), reported only while the kernel source still
    # has the hash it was measured at
    tr = traffic_from_profiles(kern, a.workload)
    roofline = dict(bound="hbm", kernel=kern, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=tr["bytes"] if tr else None,
                    avg_launch_ms=round(avg, 4), algorithmic_bytes_per_launch=int(alg))
    if tr:
        roofline["traffic_source"] = (f"profiles/traffic.json: rocprofv3 FETCH_SIZE x{tr['fetch_scale']} + "
                                      f"WRITE_SIZE x{tr['write_scale']} (copy-calibrated), measured at commit "
                                      f"{tr['commit']}, not in this run")

    out = {
        "metric": METRIC,
        "value": round(a.steps / dt, 4),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {wl.CONFIGS[a.workload]}", "n": n, "nnz": nnz, "p": p,
                   "tets": w.mesh.n_tets, "seed": a.seed, "precond": f"paper (Jacobi-PCG m={a.pcg_iters})",
                   "step_rule": "bb2", "beta": w.beta},
        "roofline": roofline,
        "kernel_ms": {k: round(v[0] / v[1], 4) for k, v in timers.items() if v[1]},
    }

    if a.calibrate_copy:
        # a plain copy of known size (2 GiB read + 2 GiB written) in the same
        # process, so counter runs can scale FETCH_SIZE / WRITE_SIZE
        src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": int(src.numel() * 8), "write": int(dst.numel() * 8)}
        del src, dst
        torch.cuda.empty_cache()

    if not a.no_converge:
        ttr = {}
        log("time to residual 1e-6: plain FP64, paper preconditioner")
        ttr["fp64_paper_precond"] = plain = run_to_tol(torch, s, X0, 1e-6, params)
        log(f"  {plain}")
        log("time to residual 1e-6: mixed precision (FP32 blocks, FP64 p x p, FP64 refinement), paper preconditioner")
        # FP32 iterations until rel < 1.5e-6 (or an FP32 stall), then FP64 to 1e-6
        mparams = dict(params, precision="f32", refine_tol=1.5e-6)
        ttr["mixed_paper_precond"] = run_to_tol(torch, s, X0, 1e-6, mparams)
        log(f"  {ttr['mixed_paper_precond']}")
        ttr.update(learned_legs(torch, s, X0, mparams))
        for k, v in ttr.items():
            if k != "fp64_paper_precond" and v.get("converged") and plain["converged"]:
                v["dE_vs_fp64_Ha"] = abs(v["energy"] - plain["energy"])
        ttr["speedup_vs_fp64_paper"] = {k: round(plain["seconds"] / v["seconds"], 3)
                                        for k, v in ttr.items() if k != "fp64_paper_precond" and v.get("converged")}
        out["time_to_residual_1e-6"] = ttr
    if a.jsonl:
        log(f"per-iteration log: {a.jsonl}")
        s.set_params(tol=1e-30, **params)
        set_start(torch, s, X0)
        jsonl_log(torch, s, a.steps, a.jsonl)
    if a.study_m:
        log(f"inner-solve length study, {a.workload}: m = {a.study_m}")
        out["m_study"] = m_study(torch, a, s, X0, params)
    if a.study_p:
        log(f"block-width study, {a.workload}: p = {a.study_p}")
        out["p_study"] = p_study(torch, a, s, w, params)
    if a.study_steps:
        log(f"step-rule study, {a.workload} seeds {a.study_steps}")
        out["step_rule_study"] = step_rule_study(torch, a, params)
    if a.study_c5:
        log(f"held-out evaluation, {a.workload} seeds {a.study_c5}")
        out["c5_study"] = c5_study(torch, a, params)
    if a.energy_check > 0:
        # the precision form's energy error, both runs converged well past 1e-6
        tol = a.energy_check
        ep = dict(params, max_iter=max(a.max_iter, 4000))
        e64 = e32 = None
        if a.energy_legs in ("both", "fp64"):
            log(f"energy check at residual {tol:g}: FP64")
            e64 = run_to_tol(torch, s, X0, tol, ep)
            log(f"  {e64}")
        if a.energy_legs in ("both", "mixed"):
            log(f"energy check at residual {tol:g}: mixed precision")
            e32 = run_to_tol(torch, s, X0, tol, dict(ep, precision="f32", refine_tol=1e-5))
            log(f"  {e32}")
        out["energy_check"] = {"tol": tol, "fp64": e64, "mixed": e32,
                               "dE_Ha": abs(e32["energy"] - e64["energy"])
                               if e64 and e32 and e64["converged"] and e32["converged"] else None}
    s.close()

    if a.cpu_baseline == "auto":
        try:
            out["cpu_baseline"] = cpu_baseline(w, X0_host, a.pcg_iters, iters=2)
        except Exception as e:  # the baseline must not hide the GPU result
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
