"""Oracle: the PCAL iteration (Section 3.3, Algorithm PCAL) on a P1 discretization.

TEST INFRASTRUCTURE ONLY.

Notation follows the paper.  X is n x p (row-major), B the mass matrix, H the
Hamiltonian, Theta(M) = Diag(diag(M)), sym(A) = (A + A^T)/2.  One iteration:

  S    = X^T B X,  Lambda0 = X^T H X                        (both symmetrized)
  kkt  = ||H X - B X Lambda0||_F,  fea = ||S - I||_F          (Section 4.1)
  stop when (kkt + fea) / kkt_0 < tol                        (Section 4.1)
  Lambda = Lambda0 + Theta(X^T grad L_beta(X, Lambda0))       (eq. lambda2)
         = Lambda0 + Theta(Lambda0 - S Lambda0 + beta S (S - I))
  G    = H X - B X Lambda + beta B X (S - I)                 (gradient of eq. prob:ALM-sub)
  P_i  = T_i^{-1} G_i with T_i = L/2 - Lambda_ii B if Lambda_ii < 0, else G_i
                                                             (eq. precondition-T)
  eta  = <Y, Y> / |<S, Y>|  (BB2, Section 4.4), S = X^k - X^{k-1}
  X_i  = (X_i - P_i / eta) / || X_i - P_i / eta ||_B           (eq. PCAL-main)

Readings where the paper is silent (each also listed in the design notes):
  * Lambda_ii in T is the diagonal of the eq. lambda2 multiplier (flag
    ``precond_lambda='lambda0'`` uses (X^T H X)_ii instead);
  * T_i^{-1} G_i is computed by Jacobi-preconditioned CG from zero with a
    fixed number m of iterations;
  * with a preconditioner, Y is the difference of preconditioned gradients
    P^k - P^{k-1} (it is the paper's Y when T = I);
  * eta_0 = ||P^0||_F / ||X^0||_F unless given; BB values are clamped to
    [1e-8, 1e8] * eta_0 and a zero or non-finite <S, Y> keeps the last eta;
  * the multiplier in kkt is Lambda0 = X^T H X.
Learned forms (not in the paper): the network's output replaces the paper
preconditioner, which takes over for fallback_hold iterations when the energy
rises above the window's minimum (or maximum) or when the fallback_stall
iterates before the current one did not halve the lowest residual.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from . import native


@dataclasses.dataclass
class Params:
    beta: float = 1.0
    tol: float = 1e-8
    max_iter: int = 1000
    precond: str = "none"          # "none" | "paper" | "learned" | "graph"
    pcg_iters: int = 10
    eta0: float = 0.0              # > 0: fixed first eta
    step_rule: str = "bb2"         # "bb2" | "bb1" | "abb1" | "abb2" | "fixed"
    precond_lambda: str = "lambda2"
    lp_weights: object = None      # learned form: (W[193], norm[8]); graph form: (W[226], norm[8])
    graph_sweeps: int = 1          # graph form: damped sweeps through T (the first after the heads)
    fallback_window: int = 5
    fallback_hold: int = 20
    fallback_rule: str = "min"     # fall back when E^k exceeds the "min" or "max" of the window
    fallback_stall: int = 30       # ... or when the last fallback_stall iterates did not halve the lowest rel (<= 0: off)
    algorithm: str = "pcal"        # "pcal" (Algorithm PCAL) | "plam" (Algorithm PLAM)


@dataclasses.dataclass
class IterRecord:
    k: int
    kkt: float
    fea: float
    rel: float
    eta: float
    energy: float


def sym(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + A.T)


class LinearProblem:
    """Fixed H and B given as CSR values on one pattern."""

    def __init__(self, row_ptr, col, Hval, Bval, Lhval=None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.Hval = np.ascontiguousarray(Hval, dtype=np.float64)
        self.Bval = np.ascontiguousarray(Bval, dtype=np.float64)
        self.Lhval = None if Lhval is None else np.ascontiguousarray(Lhval, dtype=np.float64)
        self.n = self.row_ptr.shape[0] - 1

    def set_x(self, X):            # H does not depend on X
        pass

    def hx(self, X):
        return native.spmm(self.row_ptr, self.col, self.Hval, X)

    def bx(self, X):
        return native.spmm(self.row_ptr, self.col, self.Bval, X)

    def diag(self, vals):
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        return np.asarray(vals)[self.col == rows]

    def energy(self, X, S, L0):
        """Linear problem: the Rayleigh-Ritz sum tr(S^{-1} Lambda0)."""
        return float(np.trace(np.linalg.solve(S, L0)))


def chol_gs(prob, V: np.ndarray) -> np.ndarray:
    """Cholesky-based Gram-Schmidt (Section 4.2): V = X0 R with R upper
    triangular and X0^T B X0 = I."""
    SV = sym(V.T @ prob.bx(V))
    Lc = np.linalg.cholesky(SV)                  # SV = Lc Lc^T, R = Lc^T
    return sla.solve_triangular(Lc, V.T, lower=True).T


def multiplier(S: np.ndarray, L0: np.ndarray, beta: float) -> np.ndarray:
    """eq. lambda2: Lambda0 + Theta(Lambda0 - S Lambda0 + beta S (S - I))."""
    I = np.eye(S.shape[0])
    M = L0 - S @ L0 + beta * S @ (S - I)
    return L0 + np.diag(np.diag(M))


def pcg_shifted(prob, G: np.ndarray, lam: np.ndarray, iters: int) -> np.ndarray:
    """Columnwise Jacobi-PCG from zero for (L/2 - lam_l B) x_l = G_l, fixed
    number of iterations; columns are independent (eq. precondition-T)."""
    rp, col, lh, bv = prob.row_ptr, prob.col, prob.Lhval, prob.Bval
    Dg = prob.diag(lh)[:, None] - lam[None, :] * prob.diag(bv)[:, None]
    x = np.zeros_like(G)
    r = G.copy()
    z = r / Dg
    d = z.copy()
    rz = np.sum(r * z, axis=0)
    for _ in range(iters):
        q = native.shifted_spmm(rp, col, lh, bv, lam, d)
        dq = np.sum(d * q, axis=0)
        alpha = np.where(dq > 0, rz / np.where(dq > 0, dq, 1.0), 0.0)
        x += alpha * d
        r -= alpha * q
        z = r / Dg
        rz_new = np.sum(r * z, axis=0)
        bcoef = np.where(rz > 0, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
        rz = rz_new
        d = z + bcoef * d
    return x


def precondition(prob, G, lam_diag, params: Params, kind: str = None):
    kind = kind or params.precond
    if kind == "none":
        return G
    if kind == "learned":
        from . import mlp
        W, norm = params.lp_weights
        lhd = prob.diag(prob.Lhval)
        return mlp.apply(W, norm, lhd, prob.diag(prob.Bval), prob.diag(prob.Hval), lam_diag, G)
    if kind == "graph":
        # the graph form (oracle/gnn.py)
        import scipy.sparse as sp
        from . import gnn
        W, norm = params.lp_weights
        mat = lambda v: sp.csr_matrix((v, prob.col, prob.row_ptr), shape=(prob.n, prob.n))
        return gnn.apply(W, norm, mat(prob.Lhval), mat(prob.Bval), prob.diag(prob.Hval), lam_diag, G,
                         sweeps=params.graph_sweeps)
    if kind != "paper":
        raise ValueError(kind)
    neg = lam_diag < 0
    P = G.copy()
    if np.any(neg):
        idx = np.nonzero(neg)[0]
        P[:, idx] = pcg_shifted(prob, np.ascontiguousarray(G[:, idx]), lam_diag[idx],
                                params.pcg_iters)
    return P


def bb_eta(rule: str, k: int, s: np.ndarray, y: np.ndarray, eta_prev: float, eta0: float) -> float:
    sy = float(np.sum(s * y))
    yy = float(np.sum(y * y))
    ss = float(np.sum(s * s))
    if rule == "fixed":
        return eta0
    if rule == "bb1" or (rule == "abb1" and k % 2 == 1) or (rule == "abb2" and k % 2 == 0):
        num, den = abs(sy), ss
    else:
        num, den = yy, abs(sy)
    if not (den > 0 and math.isfinite(num) and math.isfinite(den)):
        return eta_prev
    eta = num / den
    if not (eta > 0 and math.isfinite(eta)):
        return eta_prev
    return min(max(eta, 1e-8 * eta0), 1e8 * eta0)


def pcal(prob, X0: np.ndarray, params: Params,
         callback: Optional[Callable] = None, return_state: bool = False):
    """Run PCAL (or PLAM, params.algorithm) from X0 (B-orthonormal).  Returns X^k
    and the per-iteration log."""
    X = np.array(X0, dtype=np.float64, copy=True)
    p = X.shape[1]
    I = np.eye(p)
    hist: List[IterRecord] = []
    Xprev = Pprev = None
    eta = eta0 = None
    kkt0 = None
    ehist: List[float] = []
    hold = 0
    last_kind = None
    for k in range(params.max_iter + 1):
        prob.set_x(X)
        HX = prob.hx(X)
        BX = prob.bx(X)
        S = sym(X.T @ BX)
        L0 = sym(X.T @ HX)
        kkt = float(np.linalg.norm(HX - BX @ L0))
        fea = float(np.linalg.norm(S - I))
        if kkt0 is None:
            kkt0 = kkt
        rel = (kkt + fea) / kkt0 if kkt0 > 0 else kkt + fea   # stationary start: absolute
        E = prob.energy(X, S, L0)
        hist.append(IterRecord(k, kkt, fea, rel, float("nan") if eta is None else eta, E))
        if callback is not None:
            callback(k, X, HX, BX, S, L0)
        if rel < params.tol or k == params.max_iter:
            break
        # PLAM: Lambda = X^T H X (eq. multi); PCAL: eq. lambda2
        Lam = L0 if params.algorithm == "plam" else multiplier(S, L0, params.beta)
        G = HX + BX @ (params.beta * (S - I) - Lam)
        lam_diag = np.diag(Lam) if params.precond_lambda == "lambda2" else np.diag(L0)
        kind = params.precond
        if params.precond in ("learned", "graph"):
            # fall back to the paper preconditioner for fallback_hold steps when
            # E^k exceeds the minimum (or maximum) of the previous
            # fallback_window energies (fallback_window <= 0: never), or when the
            # fallback_stall iterates before this one did not halve the lowest
            # residual (a stall while the energy still falls; <= 0: never)
            use_learned = hold == 0
            if params.fallback_window > 0:
                ref = (max if params.fallback_rule == "max" else min)(ehist) if ehist else None
                if use_learned and ehist and E > ref + 1e-12 * abs(E):
                    hold = max(1, params.fallback_hold)
                    use_learned = False
                ehist = (ehist + [E])[-params.fallback_window:]
            if use_learned and params.fallback_stall > 0 and k > params.fallback_stall:
                prev = [h.rel for h in hist[:-1]]       # rel of X^0 .. X^(k-1)
                if min(prev) > 0.5 * min(prev[:k - params.fallback_stall]):
                    hold = max(1, params.fallback_hold)
                    use_learned = False
            kind = params.precond if use_learned else "paper"
            if hold > 0 and not use_learned:
                hold -= 1
        P = precondition(prob, G, lam_diag.copy(), params, kind)
        if not np.any(P):
            break                                  # P = 0: X is a fixed point of the update
        if k == 0:
            eta0 = params.eta0 if params.eta0 > 0 else float(np.linalg.norm(P) / np.linalg.norm(X))
            eta = eta0
        elif kind != last_kind:
            pass                                   # BB history restarts; eta carries over
        else:
            eta = bb_eta(params.step_rule, k, X - Xprev, P - Pprev, eta, eta0)
        last_kind = kind
        Xt = X - P / eta
        if params.algorithm == "plam":             # eq. PLAM-main: no normalization
            Xprev, Pprev = X, P
            X = Xt
            continue
        dn = np.sqrt(np.einsum("ij,ij->j", Xt, prob.bx(Xt)))
        Xprev, Pprev = X, P
        X = Xt / dn
    if return_state:
        return X, hist, dict(S=S, L0=L0, HX=HX, BX=BX)
    return X, hist


def rayleigh_ritz(prob, X: np.ndarray):
    """Post-processing (Section 4.3): solve Lambda0 y = lambda S y (p x p) and
    rotate X <- X Y.  Returns (eigenvalues ascending, rotated X)."""
    prob.set_x(X)
    S = sym(X.T @ prob.bx(X))
    L0 = sym(X.T @ prob.hx(X))
    lam, Y = sla.eigh(L0, S)
    return lam, X @ Y
