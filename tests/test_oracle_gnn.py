"""Pins of the oracle's graph (message-passing) learned preconditioner:
backpropagation against central differences, the two special cases that
reduce to the Jacobi of T and to two Jacobi sweeps written out with scipy, and
the training objective against an exact solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import fem, gnn, mlp, pcal

LAM = np.array([-0.7, 0.25, -2.0])        # column 1 takes the identity branch


@pytest.fixture(scope="module")
def c1():
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    prob = pcal.LinearProblem(d.row_ptr, d.col, d.H, d.B, 0.5 * d.L)
    Lh, Bm = d.csr(0.5 * d.L), d.csr(d.B)
    hd = prob.diag(d.H)
    G = np.random.default_rng(31).standard_normal((d.n, len(LAM)))
    return Lh, Bm, hd, G


def _norm():
    return np.array([1.0, -5.0, -2.0, 0.0, 1.0, 2.0, 3.0, 1.0])


def _trained_like(seed):
    """Weights with a non-zero output layer, so both heads act."""
    W = gnn.init_weights(seed)
    rng = np.random.default_rng(seed + 100)
    W[5 * gnn.H:] = rng.standard_normal(2 * gnn.H + 2) * 0.15
    return W


def test_gnn_backprop_matches_central_differences(c1):
    Lh, Bm, hd, G = c1
    W, norm = _trained_like(2), _norm()
    loss, g = gnn.loss_grad(W, norm, Lh, Bm, hd, LAM, G)
    rng = np.random.default_rng(9)
    picks = np.concatenate([rng.choice(5 * gnn.H, 12, replace=False),
                            5 * gnn.H + rng.choice(2 * gnn.H + 2, 12, replace=False)])
    for k in picks:
        e = np.zeros(gnn.NPAR)
        h = 1e-6
        e[k] = h
        fd = (gnn.loss_grad(W + e, norm, Lh, Bm, hd, LAM, G)[0]
              - gnn.loss_grad(W - e, norm, Lh, Bm, hd, LAM, G)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_gnn_zero_output_layer_is_the_jacobi_of_T(c1):
    """exp(0) = 1 and ft = 0: P = J G, the untrained pointwise form."""
    Lh, Bm, hd, G = c1
    W = gnn.init_weights(4)
    P = gnn.apply(W, _norm(), Lh, Bm, hd, LAM, G)
    lhd, bd = Lh.diagonal(), Bm.diagonal()
    assert np.allclose(P[:, 0], G[:, 0] / (lhd + 0.7 * bd), rtol=1e-14)
    assert np.array_equal(P[:, 1], G[:, 1])
    assert np.allclose(P[:, 2], G[:, 2] / (lhd + 2.0 * bd), rtol=1e-14)
    Pm = mlp.apply(mlp.init_weights(4), _norm(), lhd, bd, hd, LAM, G)
    assert np.allclose(P, Pm, rtol=1e-14)


def test_gnn_unit_heads_are_two_jacobi_sweeps(c1):
    """fs = 0, ft = 1 (zero output weights, biases 0 and 1): P = P1 + D^-1 (G -
    T P1) with P1 = D^-1 G, D = diag(T), written out with scipy per column."""
    Lh, Bm, hd, G = c1
    W = gnn.init_weights(5)
    W[-2:] = [0.0, 1.0]
    P = gnn.apply(W, _norm(), Lh, Bm, hd, LAM, G)
    for l, lam in enumerate(LAM):
        T = (Lh - lam * Bm) if lam < 0 else None
        if T is None:
            # T = I: the first sweep is exact, the second adds nothing
            assert np.allclose(P[:, l], G[:, l], rtol=1e-14)
            continue
        dinv = 1.0 / T.diagonal()
        p1 = dinv * G[:, l]
        p2 = p1 + dinv * (G[:, l] - T @ p1)
        assert np.allclose(P[:, l], p2, rtol=1e-12, atol=1e-14 * np.abs(p2).max())
        # and the sweep moves toward the solve: a smaller T-norm error than p1
        t = spla.spsolve(T.tocsc(), G[:, l])
        err = lambda v: float((v - t) @ (T @ (v - t)))
        assert err(p2) < err(p1)


def test_gnn_loss_is_the_T_norm_error_up_to_the_solve_energy(c1):
    """loss = sum_l w_l (||P_l - T_l^-1 G_l||_T^2 - G_l^T T_l^-1 G_l) / 2 with
    w_l = 1 / G_l^T J_l G_l, checked against a direct solve."""
    Lh, Bm, hd, G = c1
    W, norm = _trained_like(6), _norm()
    loss, _ = gnn.loss_grad(W, norm, Lh, Bm, hd, LAM, G)
    P = gnn.apply(W, norm, Lh, Bm, hd, LAM, G)
    J = mlp.jacobi(Lh.diagonal(), Bm.diagonal(), LAM)
    ref = 0.0
    for l, lam in enumerate(LAM):
        T = (Lh - lam * Bm) if lam < 0 else None
        t = spla.spsolve(T.tocsc(), G[:, l]) if T is not None else G[:, l]
        e = P[:, l] - t
        tn = float(e @ (T @ e)) if T is not None else float(e @ e)
        ref += (tn - float(G[:, l] @ t)) / 2.0 / float(G[:, l] @ (J[:, l] * G[:, l]))
    assert abs(loss - ref) <= 1e-10 * abs(ref)


def test_gnn_gradient_step_lowers_the_loss(c1):
    Lh, Bm, hd, G = c1
    W, norm = _trained_like(7), _norm()
    loss, g = gnn.loss_grad(W, norm, Lh, Bm, hd, LAM, G)
    step = 1e-3 / max(1.0, float(np.linalg.norm(g)))
    assert gnn.loss_grad(W - step * g, norm, Lh, Bm, hd, LAM, G)[0] < loss


def test_gnn_sweeps_converge_to_the_solve_of_T(c1):
    """Repeated damped sweeps with fixed heads (fs = 0, ft = 0.65) are
    Richardson iteration on T_l x = g_l with the Jacobi weights, P_m -> T_l^-1
    g_l (eq. precondition-T): the T-norm error falls with every doubling of
    the sweeps and reaches rounding (a direct solve by scipy is the
    reference); identity-branch columns stay g_l.  Two sweeps equal the
    recurrence written out with scipy matrices."""
    Lh, Bm, hd, G = c1
    W = gnn.init_weights(0)
    W[5 * gnn.H:] = 0.0
    W[-1] = 0.65                         # b2 = (fs, ft) = (0, 0.65)
    norm = _norm()
    Ts = [(Lh - l * Bm).tocsc() for l in LAM]
    X = np.column_stack([spla.spsolve(Ts[i], G[:, i]) if l < 0 else G[:, i] for i, l in enumerate(LAM)])
    J = mlp.jacobi(Lh.diagonal(), Bm.diagonal(), LAM)

    def tnorm_err(P):
        return [float(np.sqrt((P[:, i] - X[:, i]) @ (Ts[i] @ (P[:, i] - X[:, i])))) for i in (0, 2)]

    prev = None
    for m in (1, 2, 4, 16, 64, 256):
        P = gnn.apply(W, norm, Lh, Bm, hd, LAM, G, sweeps=m)
        assert np.array_equal(P[:, 1], G[:, 1])
        e = tnorm_err(P)
        if prev is not None:
            assert all(a < b for a, b in zip(e, prev)) or max(e) < 1e-12 * np.abs(X).max()
        prev = e
    ref = [float(np.sqrt(X[:, i] @ (Ts[i] @ X[:, i]))) for i in (0, 2)]
    assert all(a < 1e-12 * r for a, r in zip(prev, ref))
    # two sweeps written out
    P1 = J * G + 0.65 * J * (G - np.column_stack([Ts[i] @ (J[:, i] * G[:, i]) if l < 0 else J[:, i] * G[:, i]
                                                   for i, l in enumerate(LAM)]))
    TP1 = np.column_stack([Ts[i] @ P1[:, i] if l < 0 else P1[:, i] for i, l in enumerate(LAM)])
    P2 = P1 + 0.65 * J * (G - TP1)
    assert np.allclose(gnn.apply(W, norm, Lh, Bm, hd, LAM, G, sweeps=2), P2, rtol=1e-13, atol=1e-13)
