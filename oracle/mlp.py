"""Oracle: the learned pointwise preconditioner (not in the paper).

TEST INFRASTRUCTURE ONLY.

Definition (FP64 here; the library evaluates it in FP32):
  feat_il = [log(L_ii/2), log B_ii, (H_ii - L_ii/2)/B_ii, g_il / rms(g_l)]
  x       = (feat - mu) / sigma
  f       = W2 . tanh(W1 x + b1) + b2,   W1: 32 x 4, b1: 32, W2: 32, b2: scalar
  J_il    = 1 / (L_ii/2 - lambda_l B_ii) if lambda_l < 0 else 1
  P_il    = exp(f) J_il g_il
Parameter vector: [W1 row-major (128), b1 (32), W2 (32), b2 (1)] = 193 values.
Training objective over samples s = (feat, a, t, w):
  loss = sum_s w_s (exp(f_s) a_s - t_s)^2
Samples of one iterate (rows i, columns l; g = G_il, a = J_il g, t = (T_l^-1 G_l)_i):
  Euclidean imitation:    (a, t, n / sum_i t_il^2)
  energy-norm imitation:  (1, g / u, max(a u, 0) n / <G_l, T_l^-1 G_l>),  u = (T_l J_l G_l)_i
The second is the quadratic model d^T T d / 2 - g^T d of the paper's operator
T (eq. precondition-T) over d = s J g with the scale s taken as locally
constant: sum_i a_i u_i (s_i - g_i / u_i)^2 equals ||s J g - T^-1 g||_T^2 up
to a term without s when s is constant.
"""
from __future__ import annotations

import numpy as np

H = 32
NPAR = 4 * H + H + H + 1


def unpack(W: np.ndarray):
    W = np.asarray(W, dtype=np.float64)
    return W[:4 * H].reshape(H, 4), W[4 * H:5 * H], W[5 * H:6 * H], W[6 * H]


def forward(W: np.ndarray, norm: np.ndarray, feat: np.ndarray):
    """f for raw features feat [..., 4]; returns (f, hidden, standardized x)."""
    W1, b1, W2, b2 = unpack(W)
    norm = np.asarray(norm, dtype=np.float64)
    x = (feat - norm[:4]) / norm[4:]
    h = np.tanh(x @ W1.T + b1)
    return h @ W2 + b2, h, x


def node_features(lhd, bd, hd):
    return np.stack([np.log(lhd), np.log(bd), (hd - lhd) / bd], axis=1)


def features(lhd, bd, hd, G):
    """Raw features for every (i, l) of the block G (n x p) -> [n, p, 4]."""
    n, p = G.shape
    rms = np.sqrt(np.sum(G * G, axis=0) / n)
    node = node_features(lhd, bd, hd)
    F = np.empty((n, p, 4))
    F[:, :, :3] = node[:, None, :]
    F[:, :, 3] = np.where(rms > 0, G / np.where(rms > 0, rms, 1.0), 0.0)
    return F


def jacobi(lhd, bd, lam):
    """J_il of the paper's T_l (identity branch for lambda_l >= 0)."""
    lam = np.asarray(lam, dtype=np.float64)
    J = 1.0 / (lhd[:, None] - lam[None, :] * bd[:, None])
    return np.where(lam[None, :] < 0, J, 1.0)


def apply(W, norm, lhd, bd, hd, lam, G):
    f, _, _ = forward(W, norm, features(lhd, bd, hd, G))
    return np.exp(f) * jacobi(lhd, bd, lam) * G


def loss_grad(W, norm, S: np.ndarray):
    """Loss and its gradient (sums over samples S [m, 8]) by backpropagation."""
    W1, b1, W2, b2 = unpack(W)
    f, h, x = forward(W, norm, S[:, :4])
    a, t, w = S[:, 4], S[:, 5], S[:, 6]
    pa = np.exp(f) * a
    r = pa - t
    loss = float(np.sum(w * r * r))
    df = 2.0 * w * r * pa                       # dloss/df per sample
    gW2 = h.T @ df
    gb2 = float(np.sum(df))
    dz = (df[:, None] * W2[None, :]) * (1.0 - h * h)
    gW1 = dz.T @ x
    gb1 = dz.sum(axis=0)
    return loss, np.concatenate([gW1.ravel(), gb1, gW2, [gb2]])


def init_weights(seed: int) -> np.ndarray:
    """Small random first layer, zero output layer: the untrained network is
    exactly the Jacobi preconditioner of T (exp(0) = 1)."""
    rng = np.random.default_rng(seed)
    W = np.zeros(NPAR)
    W[:4 * H] = rng.standard_normal(4 * H) * 0.5
    W[4 * H:5 * H] = rng.standard_normal(H) * 0.1
    return W


def samples(lhd, bd, hd, lam, G, t, u, objective: str, clamp: bool = True):
    """Samples [n, p, 7] = (4 raw features, a, t, w) of every (row, column).
    t: the paper preconditioner's output for G; u: T (J G) columnwise (G on
    identity-branch columns).  clamp=False keeps negative energy weights (pins only)."""
    n, p = G.shape
    a = jacobi(lhd, bd, lam) * G
    F = features(lhd, bd, hd, G)
    if objective == "euclid":
        A, Tt = a, t
        W = np.broadcast_to(n / np.sum(t * t, axis=0), (n, p))
    else:
        A = np.ones((n, p))
        with np.errstate(divide="ignore", invalid="ignore"):
            Tt = np.where(u != 0, G / u, 0.0)
        au = a * u
        W = (np.maximum(au, 0.0) if clamp else au) * (n / np.sum(G * t, axis=0))[None, :]
        W = np.where(u != 0, W, 0.0)
    return np.concatenate([F, A[..., None], Tt[..., None], W[..., None]], axis=2)
