"""Pins of the oracle's learned preconditioner (forward, backward, special cases)."""
import numpy as np
import pytest

import workloads as wl
from oracle import fem, mlp, pcal


def _samples(m, seed):
    rng = np.random.default_rng(seed)
    S = np.zeros((m, 8))
    S[:, :4] = rng.standard_normal((m, 4)) * [1.0, 2.0, 3.0, 0.5] + [1.0, -5.0, -2.0, 0.0]
    S[:, 4] = rng.standard_normal(m)
    S[:, 5] = S[:, 4] * np.exp(0.3 * rng.standard_normal(m))
    S[:, 6] = rng.uniform(0.5, 2.0, m)
    return S


def test_backprop_matches_central_differences():
    W = mlp.init_weights(3)
    W[5 * mlp.H:] = np.random.default_rng(4).standard_normal(mlp.H + 1) * 0.2
    norm = np.array([1.0, -5.0, -2.0, 0.0, 1.0, 2.0, 3.0, 0.5])
    S = _samples(500, 5)
    loss, g = mlp.loss_grad(W, norm, S)
    rng = np.random.default_rng(6)
    for k in rng.choice(mlp.NPAR, 25, replace=False):
        e = np.zeros(mlp.NPAR)
        h = 1e-6
        e[k] = h
        fd = (mlp.loss_grad(W + e, norm, S)[0] - mlp.loss_grad(W - e, norm, S)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k
    # the loss is the definition written out
    f, _, _ = mlp.forward(W, norm, S[:, :4])
    assert abs(loss - np.sum(S[:, 6] * (np.exp(f) * S[:, 4] - S[:, 5]) ** 2)) < 1e-9 * loss


def test_untrained_network_is_the_jacobi_of_the_paper_operator():
    """Zero output layer: exp(f) = 1, so P = J G with J = diag(L/2 - lambda B)^-1
    for lambda < 0 and the identity otherwise (eq. precondition-T's branches)."""
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    W = mlp.init_weights(0)
    norm = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    G = np.random.default_rng(1).standard_normal((d.n, 3))
    lam = np.array([-0.7, 0.2, -2.0])
    P = mlp.apply(W, norm, prob.diag(0.5 * d.L), prob.diag(d.B), prob.diag(d.H), lam, G)
    lhd, bd = prob.diag(0.5 * d.L), prob.diag(d.B)
    assert np.allclose(P[:, 0], G[:, 0] / (lhd + 0.7 * bd), rtol=1e-14)
    assert np.array_equal(P[:, 1], G[:, 1])
    assert np.allclose(P[:, 2], G[:, 2] / (lhd + 2.0 * bd), rtol=1e-14)
    # and the node feature (H_ii - L_ii/2)/B_ii is the diagonal of M_ext over B
    F = mlp.features(lhd, bd, prob.diag(d.H), G)
    assert np.allclose(F[:, 0, 2], prob.diag(d.Mext) / bd, rtol=1e-12)


def test_learned_form_with_untrained_network_still_converges():
    """The learned form falls back to the paper preconditioner when the energy
    rises, so even a poor network reaches the dense eigenvalues."""
    import json, os
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(0, d.n, w.p))
    W = mlp.init_weights(0)
    W[-1] = 3.0                                   # poisoned: steps 20x too long
    norm = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    X, hist = pcal.pcal(prob, X0, pcal.Params(beta=w.beta, tol=1e-9, max_iter=3000, precond="learned",
                                              lp_weights=(W, norm)))
    assert hist[-1].rel < 1e-9
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_dense_eigs.json")))
    assert abs(hist[-1].energy - sum(ref["eigenvalues"][: w.p])) < 1e-8


def test_energy_samples_give_the_T_norm_error_for_a_constant_scale():
    """For a constant scale s the energy-norm samples' loss differs from
    ||s J g - T^-1 g||_T^2 (per-column weight included) by a term without s,
    so both have the minimizer s* = (J g)^T g / (J g)^T T (J g); clamping only
    drops the negative weights."""
    import scipy.sparse.linalg as spla
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    lhd, bd, hd = prob.diag(0.5 * d.L), prob.diag(d.B), prob.diag(d.H)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((d.n, 3))
    lam = np.array([-0.6, 0.3, -2.5])
    Ts = [d.csr(0.5 * d.L) - lam[l] * d.csr(d.B) if lam[l] < 0 else None for l in range(3)]
    t = np.stack([spla.spsolve(Ts[l].tocsc(), G[:, l]) if Ts[l] is not None else G[:, l] for l in range(3)], axis=1)
    a = mlp.jacobi(lhd, bd, lam) * G
    u = np.stack([Ts[l] @ a[:, l] if Ts[l] is not None else G[:, l] for l in range(3)], axis=1)
    S = mlp.samples(lhd, bd, hd, lam, G, t, u, "energy", clamp=False)
    for l in range(3):
        Tl = Ts[l] if Ts[l] is not None else None
        scale = d.n / float(G[:, l] @ t[:, l])

        def tnorm2(v):
            return float(v @ (Tl @ v)) if Tl is not None else float(v @ v)

        diffs, mags = [], []
        for sc in (0.3, 0.9, 1.7, 4.0):
            Lp = float(np.sum(S[:, l, 6] * (sc * S[:, l, 4] - S[:, l, 5]) ** 2))
            diffs.append(Lp - scale * tnorm2(sc * a[:, l] - t[:, l]))
            mags.append(abs(Lp))
        assert np.ptp(diffs) <= 1e-10 * max(mags)
        s_star = float(a[:, l] @ G[:, l]) / tnorm2(a[:, l])
        s_fit = float(np.sum(S[:, l, 6] * S[:, l, 5]) / np.sum(S[:, l, 6]))
        assert abs(s_fit - s_star) <= 1e-10 * abs(s_star)
    Sc = mlp.samples(lhd, bd, hd, lam, G, t, u, "energy")
    assert np.all(Sc[:, :, 6] >= 0)
    assert np.array_equal(Sc[:, :, 6], np.maximum(S[:, :, 6], 0.0))
    # the identity-branch column: T = I, J = 1, so every target is 1
    assert np.allclose(S[:, 1, 5], 1.0)


def test_stalled_learned_form_falls_back_by_the_stall_rule():
    """A network whose scale depends strongly on the residual feature makes
    the preconditioned step nonlinear in G: BB crawls (rel still ~3e-2 after
    600 iterations) while the energy does not rise, so the energy rule never
    fires.  The stall rule (the last S iterates did not halve the lowest
    residual) hands the iteration to the paper preconditioner for
    fallback_hold steps at a time, and the run converges."""
    import json, os
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    X0 = pcal.chol_gs(prob, wl.random_block(0, d.n, w.p))
    W = np.zeros(mlp.NPAR)
    W[3] = 3.0                 # hidden unit 0 reads the residual feature
    W[5 * mlp.H] = 3.0         # and drives the log-scale
    norm = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    prm = dict(beta=w.beta, tol=1e-9, max_iter=600, precond="learned", lp_weights=(W, norm), fallback_window=0)
    _, stuck = pcal.pcal(prob, X0, pcal.Params(fallback_stall=0, **prm))
    assert len(stuck) == 601 and stuck[-1].rel > 1e-2
    _, hist = pcal.pcal(prob, X0, pcal.Params(fallback_stall=10, **prm))
    assert hist[-1].rel < 1e-9
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_dense_eigs.json")))
    assert abs(hist[-1].energy - sum(ref["eigenvalues"][: w.p])) < 1e-8
