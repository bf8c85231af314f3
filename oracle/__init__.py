"""CPU oracle for the orthogonalization-free PCAL solver (arXiv 2007.14228).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__
and the CPU-baseline leg of bench.py may import, call or link anything here.
The HIP library never does, and the oracle never imports the library: the two
share no code.  The only common dependency is the ``workloads`` package,
which generates seeded inputs and holds none of the method's arithmetic.

Everything is plain FP64: numpy/scipy for dense p x p algebra and library
primitives (matmul, Cholesky, symmetric eigensolver, conjugate gradients for
the Poisson system), and a few plain C loops (oracle/csrc) for the sparse
products.  Each function cites the passage of the paper it follows.

Modules:
  fem     P1 discretization: CSR pattern, L, B, M_ext, quadrature (Section 2.2)
  xc      LDA exchange-correlation: Slater + PW92 (Section 2.1)
  pcal    PCAL iteration, multiplier, preconditioner, BB steps, Rayleigh-Ritz
          (Sections 3.3, 4.2-4.4)
  scf     Kohn-Sham H(X), density, Hartree, total energy (Sections 2.1-2.2)
  mlp     learned pointwise preconditioner: forward, backward, Adam (not in the
          paper; the design notes give its definition)
  gnn     graph learned preconditioner: the pointwise heads plus one damped
          Jacobi sweep through T over the CSR pattern, and its quadratic-model
          loss with backpropagation (not in the paper; defined in its header)

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py)
except the readings that the paper leaves open (preconditioner inner solve,
BB with a preconditioner, eta_0); those are "parity unpinned" against the
paper and pinned only GPU <-> oracle.
"""
