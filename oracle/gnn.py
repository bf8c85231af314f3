"""Oracle: the graph (message-passing) learned preconditioner (not in the paper).

TEST INFRASTRUCTURE ONLY.

A pointwise network gives every (row i, column l) a scale and a smoothing
weight; one message-passing layer over the CSR pattern, a damped Jacobi sweep
through the paper's operator T_l (eq. precondition-T), then smooths.  A
pointwise rescaling cannot represent T_l^-1, which amplifies smooth
components; the sweep can.

Definition (FP64):
  feat_il  = the four features of the pointwise form (oracle/mlp.py)
  x        = (feat - mu) / sigma
  (fs, ft) = W2 tanh(W1 x + b1) + b2,   W1: 32 x 4, b1: 32, W2: 2 x 32, b2: 2
  T_l      = L/2 - lambda_l B if lambda_l < 0, else the identity
  J_l      = the Jacobi of T_l (oracle/mlp.py: jacobi)
  Z_l      = exp(fs_l) J_l G_l
  R_l      = G_l - T_l Z_l                           (the SpMM-shaped layer)
  P_l      = Z_l + ft_l J_l R_l
Special cases: a zero output layer gives P = J G, the untrained pointwise
form; fs = 0, ft = 1 give two Jacobi sweeps on T_l P_l = G_l from zero.
Parameter vector: [W1 row-major (128), b1 (32), W2 row-major (64), b2 (2)] =
226 values.

Training objective, which needs no solve with T_l: the quadratic model of
each column's system,
  loss = sum_l w_l (P_l^T T_l P_l / 2 - G_l^T P_l),   w_l = 1 / (G_l^T J_l G_l),
equal to sum_l w_l (||P_l - T_l^-1 G_l||_T^2 - G_l^T T_l^-1 G_l) / 2, so it
is smallest where P_l is the paper preconditioner's exact output.
"""
from __future__ import annotations

import numpy as np

from . import mlp

H = mlp.H
NPAR = 4 * H + H + 2 * H + 2


def unpack(W: np.ndarray):
    W = np.asarray(W, dtype=np.float64)
    return (W[:4 * H].reshape(H, 4), W[4 * H:5 * H], W[5 * H:7 * H].reshape(2, H), W[7 * H:7 * H + 2])


def init_weights(seed: int) -> np.ndarray:
    """Small random first layer, zero output layer: the untrained network is
    the Jacobi of T, as for the pointwise form."""
    rng = np.random.default_rng(seed)
    W = np.zeros(NPAR)
    W[:4 * H] = rng.standard_normal(4 * H) * 0.5
    W[4 * H:5 * H] = rng.standard_normal(H) * 0.1
    return W


def heads(W: np.ndarray, norm: np.ndarray, F: np.ndarray):
    """(fs, ft) for raw features F [..., 4]; also the hidden layer and x."""
    W1, b1, W2, b2 = unpack(W)
    norm = np.asarray(norm, dtype=np.float64)
    x = (F - norm[:4]) / norm[4:]
    h = np.tanh(x @ W1.T + b1)
    out = h @ W2.T + b2
    return out[..., 0], out[..., 1], h, x


def operators(Lh, Bm, lam):
    """T_l as sparse matrices (None: the identity branch)."""
    return [Lh - float(l) * Bm if l < 0 else None for l in np.asarray(lam, dtype=np.float64)]


def _apply_T(Ts, V):
    """Columnwise T_l v_l."""
    out = np.empty_like(V)
    for l, T in enumerate(Ts):
        out[:, l] = T @ V[:, l] if T is not None else V[:, l]
    return out


def _forward(W, norm, Lh, Bm, hd, lam, G):
    lhd, bd = Lh.diagonal(), Bm.diagonal()
    fs, ft, h, x = heads(W, norm, mlp.features(lhd, bd, hd, G))
    J = mlp.jacobi(lhd, bd, lam)
    Ts = operators(Lh, Bm, lam)
    Z = np.exp(fs) * J * G
    R = G - _apply_T(Ts, Z)
    P = Z + ft * J * R
    return dict(fs=fs, ft=ft, h=h, x=x, J=J, Ts=Ts, Z=Z, R=R, P=P)


def apply(W, norm, Lh, Bm, hd, lam, G, sweeps: int = 1):
    """P for the block G (n x p); Lh = L/2 and Bm = B as scipy sparse
    matrices, hd the diagonal of H.  sweeps > 1 repeats the damped sweep
    with the same weights, P <- P + ft J (G - T P): a fixed polynomial in
    J T applied to G, which for 0 < ft J T < 2 tends to T^-1 G (the
    preconditioner of eq. precondition-T) as the sweeps grow."""
    f = _forward(W, norm, Lh, Bm, hd, lam, G)
    P = f["P"]
    for _ in range(sweeps - 1):
        P = P + f["ft"] * f["J"] * (G - _apply_T(f["Ts"], P))
    return P


def loss_grad(W, norm, Lh, Bm, hd, lam, G):
    """The quadratic-model loss and its gradient by backpropagation through
    the sweep (T_l is symmetric) and the two heads."""
    f = _forward(W, norm, Lh, Bm, hd, lam, G)
    J, Ts, Z, R, P, ft, h, x = f["J"], f["Ts"], f["Z"], f["R"], f["P"], f["ft"], f["h"], f["x"]
    w = 1.0 / np.sum(G * J * G, axis=0)
    TP = _apply_T(Ts, P)
    loss = float(np.sum(w * (0.5 * np.sum(P * TP, axis=0) - np.sum(G * P, axis=0))))
    dP = w[None, :] * (TP - G)                  # d loss / d P
    dft = dP * J * R
    dR = ft * J * dP
    dZ = dP - _apply_T(Ts, dR)                  # R = G - T Z
    dfs = dZ * Z                                # Z = exp(fs) J G
    _, _, W2, _ = unpack(W)
    dout = np.stack([dfs, dft], axis=-1)        # [n, p, 2]
    gW2 = np.einsum("ipk,iph->kh", dout, h)
    gb2 = dout.sum(axis=(0, 1))
    dz = (dout @ W2) * (1.0 - h * h)
    gW1 = np.einsum("ipj,ipc->jc", dz, x)
    gb1 = dz.sum(axis=(0, 1))
    return loss, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])
