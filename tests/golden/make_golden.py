"""Writes the stored expected values under tests/golden/.

Calls only the oracle (and LAPACK through scipy for the dense reference).
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import fem  # noqa: E402


def c1_dense_eigs():
    """Eight smallest eigenvalues of the generalized problem H x = lambda B x of
    the 16^3-cell workload (dense LAPACK, the brute-force pin of Section 4.3's
    post-processing)."""
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    ev = sla.eigh(d.csr(d.H).toarray(), d.csr(d.B).toarray(), eigvals_only=True,
                  subset_by_index=[0, 7])
    out = dict(workload=wl.CONFIGS["c1"], n=d.n, nnz=d.nnz, eigenvalues=[float(x) for x in ev],
               source="oracle discretization + scipy.linalg.eigh (LAPACK dsygvd)")
    with open(os.path.join(HERE, "c1_dense_eigs.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    c1_dense_eigs()
