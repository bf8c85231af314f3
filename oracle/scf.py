"""Oracle: the Kohn-Sham Hamiltonian H(X) and total energy (Sections 2.1-2.2).

TEST INFRASTRUCTURE ONLY.

For X (n x p, interior DOFs) and occupation f (two electrons per orbital,
Section 4.1):
  psi_l(q) = sum_a X_{v_a, l} lambda_a(q)     at the 4 quadrature points of each K
  rho(q)   = f sum_l psi_l(q)^2               (density, Section 2.2)
  b_i      = sum_K sum_q |K|/4 rho(q) lambda_i(q)
  L U      = 4 pi b                           (Hartree potential by the Poisson equation)
  V_H(q)   = sum_a U_{v_a} lambda_a(q)
  H(X)     = L/2 + M(V_ext + V_H + v_xc(rho))  (eq. hamiltonian)
  E_KS     = f tr(X^T L X)/2 + f tr(X^T M_ext X) + U.b/2 + sum_q w eps_xc rho + E_nuc
                                              (discrete energies, Section 2.2)
Readings: f = 2 on all p orbitals; zero Dirichlet data for U on the box
boundary; the Poisson system is solved by conjugate gradients to a relative
residual of 1e-12.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, native
from .pcal import LinearProblem, sym
from .xc import lda_xc


class KSProblem(LinearProblem):
    """H depends on X; ``set_x`` rebuilds H(X) before each use."""

    def __init__(self, disc: fem.Discretization, Z, R, f: float = 2.0,
                 poisson_rtol: float = 1e-12):
        super().__init__(disc.row_ptr, disc.col, disc.H, disc.B, 0.5 * disc.L)
        self.disc = disc
        self.f = f
        self.Enuc = fem.nuclear_repulsion(Z, R)
        self.poisson_rtol = poisson_rtol
        self.Lcsr = disc.csr(disc.L)
        self.Ldiag = self.diag(disc.L)
        self.U = np.zeros(disc.n)
        self.parts = None

    # -- density ------------------------------------------------------------
    def psi_q(self, X: np.ndarray) -> np.ndarray:
        d = self.disc
        dv = d.dof[d.tets]                                  # [nt, 4]
        Xe = np.where((dv >= 0)[:, :, None], X[np.maximum(dv, 0)], 0.0)   # [nt, 4, p]
        return np.einsum("qa,kal->kql", fem.BARY, Xe)       # [nt, 4, p]

    def density(self, X: np.ndarray) -> np.ndarray:
        psi = self.psi_q(X)
        return self.f * np.einsum("kql,kql->kq", psi, psi)

    def load_vector(self, rho_q: np.ndarray) -> np.ndarray:
        """b_i = int rho phi_i by the element rule."""
        d = self.disc
        w = d.vol[:, None] / 4.0 * rho_q                    # [nt, 4]
        loc = np.einsum("kq,qa->ka", w, fem.BARY)           # [nt, 4]
        dv = d.dof[d.tets].ravel()
        m = dv >= 0
        return np.bincount(dv[m], weights=loc.ravel()[m], minlength=d.n)

    def hartree(self, b: np.ndarray) -> np.ndarray:
        rhs = 4.0 * math.pi * b
        Minv = spla.LinearOperator(self.Lcsr.shape, matvec=lambda v: v / self.Ldiag)
        U, info = spla.cg(self.Lcsr, rhs, x0=self.U, rtol=self.poisson_rtol, atol=0.0,
                          M=Minv, maxiter=100000)
        if info != 0:
            raise RuntimeError(f"Poisson CG did not converge (info={info})")
        self.U = U
        return U

    def nodal_to_q(self, U: np.ndarray) -> np.ndarray:
        d = self.disc
        dv = d.dof[d.tets]
        Ue = np.where(dv >= 0, U[np.maximum(dv, 0)], 0.0)   # [nt, 4]
        return Ue @ fem.BARY.T                              # [nt, q]

    # -- Hamiltonian --------------------------------------------------------
    def build(self, X: np.ndarray):
        rho = self.density(X)
        Hval, U, parts = self.hamiltonian_from_density(rho)
        return Hval, rho, U, parts

    def hamiltonian_from_density(self, rho: np.ndarray):
        """H = L/2 + M(V_ext + V_H[rho] + v_xc(rho)) and the density-only
        energy terms."""
        d = self.disc
        b = self.load_vector(rho)
        U = self.hartree(b)
        VH = self.nodal_to_q(U)
        eps, vxc = lda_xc(rho)
        Veff = d.Vext_q + VH + vxc
        Hval = 0.5 * d.L + d.potential_matrix(Veff)
        w = d.vol[:, None] / 4.0
        parts = dict(
            har=0.5 * float(U @ b),
            xc=float(np.sum(w * eps * rho)),
            int_vxc_rho=float(np.sum(w * vxc * rho)),
            nelec=float(np.sum(w * rho)),
            nuc=self.Enuc,
        )
        return Hval, U, parts

    def set_x(self, X):
        self.Hval, self.rho, _, self.parts = self.build(X)

    def energy_direct(self, X: np.ndarray) -> dict:
        """Each term of E_KS evaluated from its own definition at X."""
        d = self.disc
        Hval, rho, U, parts = self.build(X)
        LX = native.spmm(self.row_ptr, self.col, d.L, X)
        MX = native.spmm(self.row_ptr, self.col, d.Mext, X)
        kin = self.f * 0.5 * float(np.sum(X * LX))
        ext = self.f * float(np.sum(X * MX))
        tot = kin + ext + parts["har"] + parts["xc"] + parts["nuc"]
        return dict(kin=kin, ext=ext, har=parts["har"], xc=parts["xc"], nuc=parts["nuc"],
                    total=tot, nelec=parts["nelec"])

    def energy(self, X, S, L0):
        """Double-counting form, valid at any X with H = H(X):
        E = f tr(X^T H X) - U.b/2 - int v_xc rho + int eps_xc rho + E_nuc."""
        pr = self.parts
        return (self.f * float(np.trace(L0)) - pr["har"] - pr["int_vxc_rho"] + pr["xc"]
                + pr["nuc"])

    def gradient(self, X: np.ndarray) -> np.ndarray:
        """dE_KS/dX = 2 f H(X) X (the unscaled gradient, Section 2.2)."""
        Hval, _, _, _ = self.build(X)
        return 2.0 * self.f * native.spmm(self.row_ptr, self.col, Hval, X)
