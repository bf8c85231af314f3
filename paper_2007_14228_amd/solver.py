"""Python binding of the ofks C ABI: argument marshalling only.

Every computation runs in libofks.so.  Device buffers are torch tensors on
the current HIP device; the solver is bound to the current torch stream.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import _lib
from ._lib import IterStats, Params


class OfksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ofks error {code}: {msg}")
        self.code = code


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_block(X, n: int):
    if X.dim() != 2 or int(X.shape[0]) != n or int(X.shape[1]) < 1:
        raise ValueError(f"expected an n x p block with n = {n}, got {tuple(X.shape)}")


def _dev_ptr(t, dtype_name: str = "float64"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (HIP) torch tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected torch.{dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One ofks context on the current torch HIP stream."""

    def __init__(self, stream=None):
        import torch
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.ofks_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream)), ctx=None)
        self.h = h
        self.p = 0
        self.n = 0
        self.n_tets = 0
        self.params = self.default_params()

    # -- plumbing ----------------------------------------------------------
    def _check(self, rc: int, ctx="self"):
        if rc < 0 or (rc > 0 and rc != _lib.OFKS_NOT_CONVERGED):
            msg = ""
            if ctx is not None and getattr(self, "h", None) is not None:
                msg = self.lib.ofks_last_error(self.h).decode()
            raise OfksError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ofks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def default_params(self) -> Params:
        p = Params()
        self.lib.ofks_default_params(ctypes.byref(p))
        return p

    # -- discretization ----------------------------------------------------
    def mesh_load(self, xyz: np.ndarray, tets: np.ndarray, dirichlet: np.ndarray):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        self._check(self.lib.ofks_mesh_load(self.h, xyz.shape[0], _np_ptr(xyz), tets.shape[0], _np_ptr(tets),
                                            _np_ptr(dirichlet)))
        self.n_tets = int(tets.shape[0])

    def nuclei_set(self, Z: np.ndarray, R: np.ndarray):
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, 3)
        self._check(self.lib.ofks_nuclei_set(self.h, int(Z.shape[0]), _np_ptr(Z), _np_ptr(R)))

    def assemble(self):
        self._check(self.lib.ofks_assemble(self.h))
        self.n, self.nnz = self.csr_info()

    def load_workload(self, w):
        """Mesh + nuclei + device assembly for a workloads.Workload."""
        self.mesh_load(w.mesh.xyz, w.mesh.tets, w.mesh.dirichlet)
        self.nuclei_set(w.Z, w.R)
        self.assemble()

    def csr_info(self) -> Tuple[int, int]:
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        self._check(self.lib.ofks_csr_info(self.h, ctypes.byref(n), ctypes.byref(nnz)))
        return int(n.value), int(nnz.value)

    def csr_get(self, values: bool = True) -> Dict[str, np.ndarray]:
        n, nnz = self.csr_info()
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        out = dict(row_ptr=rp, col=col)
        L = B = H = None
        if values:
            L = np.empty(nnz)
            B = np.empty(nnz)
            H = np.empty(nnz)
            out.update(L=L, B=B, H=H)
        nul = ctypes.c_void_p(None)
        self._check(self.lib.ofks_csr_get(self.h, _np_ptr(rp), _np_ptr(col),
                                          _np_ptr(L) if L is not None else nul,
                                          _np_ptr(B) if B is not None else nul,
                                          _np_ptr(H) if H is not None else nul))
        return out

    def csr_load(self, row_ptr, col, H, B, Lhalf=None):
        n = int(row_ptr.shape[0] - 1)
        nnz = int(col.shape[0])
        rp_h = row_ptr.cpu().numpy()
        col_h = col.cpu().numpy()
        if rp_h[0] != 0 or rp_h[-1] != nnz or np.any(np.diff(rp_h) < 0):
            raise ValueError("row_ptr is not a valid CSR offset array")
        if nnz and (col_h.min() < 0 or col_h.max() >= n):
            raise ValueError("column index out of range")
        for v in (H, B) + ((Lhalf,) if Lhalf is not None else ()):
            if int(v.shape[0]) != nnz:
                raise ValueError("value arrays must have nnz entries")
        self._check(self.lib.ofks_csr_load(self.h, n, nnz, _dev_ptr(row_ptr, "int64"), _dev_ptr(col, "int32"),
                                           _dev_ptr(H), _dev_ptr(B),
                                           _dev_ptr(Lhalf) if Lhalf is not None else ctypes.c_void_p(None)))
        self.n, self.nnz = n, nnz

    # -- setup ---------------------------------------------------------------
    def set_params(self, **kw):
        p = self.default_params()
        for k, v in kw.items():
            if k == "precond" and isinstance(v, str):
                v = _lib.PRECOND[v]
            elif k == "step_rule" and isinstance(v, str):
                v = _lib.STEP[v]
            elif k == "precision" and isinstance(v, str):
                v = _lib.PRECISION[v]
            elif k == "algorithm" and isinstance(v, str):
                v = {"pcal": 0, "plam": 1}[v]
            elif k == "spmm_mode" and isinstance(v, str):
                v = {"auto": 0, "gather": 1, "halo": 2}[v]
            elif k == "fallback_rule" and isinstance(v, str):
                v = {"min": 0, "max": 1}[v]
            elif k == "precond_lambda" and isinstance(v, str):
                v = {"lambda2": 0, "lambda0": 1}[v]
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        self._check(self.lib.ofks_set_params(self.h, ctypes.byref(p)))
        self.params = p

    def workspace_size(self, p: int) -> int:
        nb = ctypes.c_size_t()
        self._check(self.lib.ofks_workspace_size(self.h, int(p), ctypes.byref(self.params), ctypes.byref(nb)))
        return nb.value

    def set_workspace(self, buf):
        """buf: a device uint8 tensor that holds the iteration state from now
        on (None: back to library allocation)."""
        if buf is None:
            self._check(self.lib.ofks_set_workspace(self.h, None, 0))
            self._ws = None
            return
        self._ws = buf
        self._check(self.lib.ofks_set_workspace(self.h, ctypes.c_void_p(buf.data_ptr()), int(buf.numel())))

    def set_x0(self, X0, orthonormalize: bool = True):
        _check_block(X0, self.n)
        p = int(X0.shape[1])
        self._check(self.lib.ofks_set_x0(self.h, p, _dev_ptr(X0), 1 if orthonormalize else 0))
        self.p = p

    # -- iteration -----------------------------------------------------------
    def step(self, max_steps: int = 1) -> Tuple[List[dict], bool, int]:
        buf = (IterStats * max(1, max_steps))()
        ns = ctypes.c_int32()
        done = ctypes.c_int32()
        rc = self._check(self.lib.ofks_step(self.h, max_steps, buf, ctypes.byref(ns), ctypes.byref(done)))
        out = []
        for i in range(ns.value):
            s = buf[i]
            out.append({f: getattr(s, f) for f, _ in IterStats._fields_})
        return out, bool(done.value), rc

    def residual(self) -> Tuple[float, float, float]:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.ofks_residual(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def energy(self) -> np.ndarray:
        parts = np.empty(8)
        self._check(self.lib.ofks_energy(self.h, _np_ptr(parts)))
        return parts

    def postprocess(self) -> np.ndarray:
        eig = np.empty(self.p)
        self._check(self.lib.ofks_postprocess(self.h, _np_ptr(eig)))
        return eig

    def get_x(self):
        import torch
        X = torch.empty((self.n, self.p), dtype=torch.float64, device="cuda")
        self._check(self.lib.ofks_get_x(self.h, _dev_ptr(X)))
        return X

    def get_density(self):
        import torch
        rho = torch.empty((self.n_tets, 4), dtype=torch.float64, device="cuda")
        self._check(self.lib.ofks_get_density(self.h, _dev_ptr(rho)))
        return rho

    def update_density(self):
        self._check(self.lib.ofks_update_density(self.h))

    def state_get(self):
        """The iteration state as a device uint8 tensor (checkpoint)."""
        import torch
        nb = ctypes.c_size_t()
        self._check(self.lib.ofks_state_size(self.h, ctypes.byref(nb)))
        buf = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        self._check(self.lib.ofks_state_get(self.h, ctypes.c_void_p(buf.data_ptr()), nb.value))
        return buf

    def state_set(self, buf):
        if not buf.is_cuda or buf.dtype != __import__("torch").uint8 or not buf.is_contiguous():
            raise TypeError("state must be a contiguous device uint8 tensor")
        self._check(self.lib.ofks_state_set(self.h, ctypes.c_void_p(buf.data_ptr()), int(buf.numel())))
        self.p = self.iterate_info()[0]

    def iterate_info(self):
        """(p, precision, k) of the current iterate."""
        p, prec, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.ofks_iterate_info(self.h, ctypes.byref(p), ctypes.byref(prec), ctypes.byref(k)))
        return p.value, prec.value, k.value

    # -- single kernels -------------------------------------------------------
    def spmm(self, X):
        import torch
        _check_block(X, self.n)
        HX = torch.empty_like(X)
        BX = torch.empty_like(X)
        self._check(self.lib.ofks_spmm(self.h, int(X.shape[1]), _dev_ptr(X), _dev_ptr(HX), _dev_ptr(BX)))
        return HX, BX

    def spmm_ex(self, X, op: str = "dual", lam: Optional[np.ndarray] = None):
        """op "dual": (H X, B X); op "shift": (L/2 - lam_l B) X_l on columns
        with lam_l < 0 (zero elsewhere).  The precision follows X's dtype
        (float64 or float32)."""
        import torch
        _check_block(X, self.n)
        prec = {torch.float64: 0, torch.float32: 1}.get(X.dtype)
        if prec is None:
            raise TypeError("X must be float64 or float32")
        name = "float64" if prec == 0 else "float32"
        p = int(X.shape[1])
        Y1 = torch.empty_like(X)
        if op == "dual":
            Y2 = torch.empty_like(X)
            self._check(self.lib.ofks_spmm_ex(self.h, p, prec, 0, None, _dev_ptr(X, name), _dev_ptr(Y1, name),
                                              _dev_ptr(Y2, name)))
            return Y1, Y2
        if op != "shift":
            raise ValueError(op)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (p,):
            raise ValueError("lam must have one entry per column")
        self._check(self.lib.ofks_spmm_ex(self.h, p, prec, 1, _np_ptr(lam), _dev_ptr(X, name),
                                          _dev_ptr(Y1, name), None))
        return Y1

    def gram(self, X, HX, BX):
        for Y in (X, HX, BX):
            _check_block(Y, self.n)
        if not (X.shape == HX.shape == BX.shape):
            raise ValueError("X, HX, BX must have the same shape")
        p = int(X.shape[1])
        S = np.empty((p, p))
        L0 = np.empty((p, p))
        self._check(self.lib.ofks_gram(self.h, p, _dev_ptr(X), _dev_ptr(HX), _dev_ptr(BX), _np_ptr(S),
                                       _np_ptr(L0)))
        return S, L0

    def precondition(self, lam: np.ndarray, G):
        import torch
        _check_block(G, self.n)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (int(G.shape[1]),):
            raise ValueError("lam must have one entry per column")
        P = torch.empty_like(G)
        self._check(self.lib.ofks_precondition(self.h, int(G.shape[1]), _np_ptr(lam), _dev_ptr(G), _dev_ptr(P)))
        return P

    def build_hamiltonian(self, X):
        import torch
        _check_block(X, self.n)
        q = lambda: torch.empty((self.n_tets, 4), dtype=torch.float64, device="cuda")
        rho, eps, vxc = q(), q(), q()
        U = torch.empty(self.n, dtype=torch.float64, device="cuda")
        parts = np.empty(4)
        self._check(self.lib.ofks_build_hamiltonian(self.h, int(X.shape[1]), _dev_ptr(X), _dev_ptr(rho),
                                                    _dev_ptr(eps), _dev_ptr(vxc), _dev_ptr(U), _np_ptr(parts)))
        return dict(rho=rho, eps=eps, vxc=vxc, U=U, parts=parts)

    # -- learned preconditioner -------------------------------------------------
    def lp_set_weights(self, w: np.ndarray, norm: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        if w.shape != (193,) or norm.shape != (8,):
            raise ValueError("weights must be 193 floats and norm 8 floats")
        self._check(self.lib.ofks_lp_set_weights(self.h, _np_ptr(w), _np_ptr(norm)))

    def lp_collect(self, buf, row_stride: int, objective: str = "energy"):
        """buf: device float32 tensor [cap, 8] (or None to stop); objective
        "euclid" (0) or "energy" (1), see ofks_lp_collect."""
        obj = {"euclid": 0, "energy": 1}[objective] if isinstance(objective, str) else int(objective)
        if buf is None:
            self._check(self.lib.ofks_lp_collect(self.h, 0, obj, ctypes.c_void_p(None), 0))
            return
        if buf.dim() != 2 or int(buf.shape[1]) != 8:
            raise ValueError("sample buffer must be [cap, 8]")
        self._check(self.lib.ofks_lp_collect(self.h, int(row_stride), obj, _dev_ptr(buf, "float32"),
                                             int(buf.shape[0])))

    def lp_collected(self) -> int:
        n = ctypes.c_int64()
        self._check(self.lib.ofks_lp_collected(self.h, ctypes.byref(n)))
        return int(n.value)

    def lp_train(self, samples, epochs: int, lr: float, w0: np.ndarray):
        m = int(samples.shape[0])
        w = np.ascontiguousarray(w0, dtype=np.float32).copy()
        norm = np.empty(8, dtype=np.float32)
        loss = np.empty(max(epochs, 1))
        self._check(self.lib.ofks_lp_train(self.h, _dev_ptr(samples, "float32"), m, int(epochs), float(lr),
                                           _np_ptr(w), _np_ptr(norm), _np_ptr(loss)))
        return w, norm, loss[:epochs]

    def lp_loss_grad(self, samples, w: np.ndarray, norm: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        loss = ctypes.c_double()
        grad = np.empty(193)
        self._check(self.lib.ofks_lp_loss_grad(self.h, _dev_ptr(samples, "float32"), int(samples.shape[0]),
                                               _np_ptr(w), _np_ptr(norm), ctypes.byref(loss), _np_ptr(grad)))
        return loss.value, grad

    def lp_apply(self, lam: np.ndarray, G):
        import torch
        _check_block(G, self.n)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (int(G.shape[1]),):
            raise ValueError("lam must have one entry per column")
        P = torch.empty_like(G)
        self._check(self.lib.ofks_lp_apply(self.h, int(G.shape[1]), _np_ptr(lam), _dev_ptr(G), _dev_ptr(P)))
        return P

    def lp_features(self, G):
        """Raw features [n, p, 4] (float32) of the learned forms for block G."""
        import torch
        _check_block(G, self.n)
        F = torch.empty((self.n, int(G.shape[1]), 4), dtype=torch.float32, device="cuda")
        self._check(self.lib.ofks_lp_features(self.h, int(G.shape[1]), _dev_ptr(G), _dev_ptr(F, "float32")))
        return F

    # -- learned graph preconditioner ------------------------------------------
    def gl_set_weights(self, w: np.ndarray, norm: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        norm = np.ascontiguousarray(norm, dtype=np.float32)
        if w.shape != (226,) or norm.shape != (8,):
            raise ValueError("graph weights: 226 values and 8 standardization constants")
        self._check(self.lib.ofks_gl_set_weights(self.h, _np_ptr(w), _np_ptr(norm)))

    def gl_apply(self, lam: np.ndarray, G):
        import torch
        _check_block(G, self.n)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (int(G.shape[1]),):
            raise ValueError("lam must have one entry per column")
        P = torch.empty_like(G)
        self._check(self.lib.ofks_gl_apply(self.h, int(G.shape[1]), _np_ptr(lam), _dev_ptr(G), _dev_ptr(P)))
        return P

    def gl_loss_grad(self, lam: np.ndarray, G):
        _check_block(G, self.n)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        loss = ctypes.c_double()
        grad = np.empty(226)
        self._check(self.lib.ofks_gl_loss_grad(self.h, int(G.shape[1]), _np_ptr(lam), _dev_ptr(G),
                                               ctypes.byref(loss), _np_ptr(grad)))
        return loss.value, grad

    def gl_capture(self, buf, every: int = 1):
        """buf: device float64 tensor [slots, n, p] (None stops capturing)."""
        if buf is None:
            self._check(self.lib.ofks_gl_capture(self.h, None, 0, 0))
            self._cap = None
            return
        if buf.dim() != 3 or int(buf.shape[1]) != self.n:
            raise ValueError("capture buffer must be [slots, n, p]")
        self._cap = buf
        self._check(self.lib.ofks_gl_capture(self.h, _dev_ptr(buf), int(buf.shape[0]), int(every)))

    def gl_captured(self, p: int):
        cnt = ctypes.c_int32()
        self._check(self.lib.ofks_gl_captured(self.h, ctypes.byref(cnt), None))
        lam = np.empty((max(cnt.value, 1), p))
        self._check(self.lib.ofks_gl_captured(self.h, ctypes.byref(cnt), _np_ptr(lam)))
        return cnt.value, lam[: cnt.value]

    def gl_train(self, G, lam: np.ndarray, epochs: int, lr: float, w: np.ndarray, adam: np.ndarray):
        """Adam over the blocks G [count, n, p] with shifts lam [count, p];
        returns (weights, optimizer state, losses [epochs, count])."""
        if G.dim() != 3 or int(G.shape[1]) != self.n:
            raise ValueError("G must be [count, n, p]")
        count, p = int(G.shape[0]), int(G.shape[2])
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (count, p):
            raise ValueError("lam must be [count, p]")
        w = np.array(w, dtype=np.float32, copy=True)
        adam = np.array(adam, dtype=np.float32, copy=True)
        if w.shape != (226,) or adam.shape != (453,):
            raise ValueError("226 weights and 453 optimizer values")
        losses = np.empty((epochs, count))
        self._check(self.lib.ofks_gl_train(self.h, p, _dev_ptr(G), _np_ptr(lam), count, int(epochs),
                                           ctypes.c_float(lr), _np_ptr(w), _np_ptr(adam), _np_ptr(losses)))
        return w, adam, losses

    def gl_feature_norm(self) -> np.ndarray:
        norm = np.empty(8, dtype=np.float32)
        self._check(self.lib.ofks_gl_feature_norm(self.h, _np_ptr(norm)))
        return norm

    # -- timing ----------------------------------------------------------------
    def timing(self, enable: bool = True):
        self._check(self.lib.ofks_timing(self.h, 1 if enable else 0))

    def timer(self, name: str) -> Tuple[float, int]:
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.ofks_timer_get(self.h, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, int(n.value)
