"""The library's host-side code and the oracle's C loops built with
AddressSanitizer and UndefinedBehaviorSanitizer on the CPU (g++/gcc, host
code only; no GPU code is built here) and run on real and adversarial inputs:
any out-of-bounds access, use after free, leak, signed overflow or other
undefined behaviour aborts the driver.  The drivers also return results that
are checked against numpy/scipy, so the sanitized builds compute the same
thing as the unsanitized ones.

Covered: the LDS-halo plan (csrc/halo_plan.hpp: build and independent check),
the dense p x p algebra (csrc/dense.hpp: Cholesky, triangular inverse, the
Jacobi eigensolver, the generalized eigenproblem, tr(S^-1 A)) and the
oracle's CSR products (oracle/csrc/oracle_kernels.c)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_14228_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")

HALO_DRIVER = r"""
#include "halo_plan.hpp"
#include <cstdio>
#include <vector>
// reads n, caps and a CSR pattern; builds and checks the plan; prints the
// two status codes and the block count
int main(int argc, char **argv) {
    FILE *f = std::fopen(argv[1], "rb");
    int64_t n; int32_t hm, rm, em;
    if (std::fread(&n, 8, 1, f) != 1 || std::fread(&hm, 4, 1, f) != 1 || std::fread(&rm, 4, 1, f) != 1 ||
        std::fread(&em, 4, 1, f) != 1) return 2;
    std::vector<int64_t> rp(n + 1);
    if (std::fread(rp.data(), 8, n + 1, f) != (size_t)(n + 1)) return 2;
    std::vector<int32_t> col(rp[n] > 0 ? rp[n] : 0);
    if (std::fread(col.data(), 4, col.size(), f) != col.size()) return 2;
    std::fclose(f);
    ofks::HaloPlan P;
    int64_t where = -7, where2 = -7;
    int32_t rc = ofks::halo_plan_build(n, rp.data(), col.data(), hm, rm, em, P, &where);
    int32_t rc2 = rc == 0 ? ofks::halo_plan_check(n, rp.data(), col.data(), hm, rm, em, P, &where2) : -99;
    std::printf("%d %d %lld\n", rc, rc2, (long long)P.nb());
    return 0;
}
"""

DENSE_DRIVER = r"""
#include "dense.hpp"
#include <cstdio>
#include <vector>
// reads p, A (p x p) and S (p x p, SPD); writes the Cholesky factor of S, its
// lower inverse, the eigenvalues of A, the generalized eigenvalues of (A, S)
// and tr(S^-1 A)
int main(int argc, char **argv) {
    FILE *f = std::fopen(argv[1], "rb");
    int32_t p;
    if (std::fread(&p, 4, 1, f) != 1) return 2;
    std::vector<double> A(p * p), S(p * p);
    if (std::fread(A.data(), 8, p * p, f) != (size_t)(p * p) || std::fread(S.data(), 8, p * p, f) != (size_t)(p * p))
        return 2;
    std::fclose(f);
    std::vector<double> L = S;
    if (!ofks::dense::cholesky(L, p)) return 3;
    std::vector<double> Li = ofks::dense::lower_inverse(L, p);
    std::vector<double> w, V, gw, Y;
    ofks::dense::sym_eig(A, p, w, V);
    if (!ofks::dense::sym_gen_eig(A, S, p, gw, Y)) return 4;
    double tr = 0.0;
    if (!ofks::dense::trace_sinv_a(S, A, p, tr)) return 5;
    FILE *g = std::fopen(argv[2], "wb");
    std::fwrite(L.data(), 8, p * p, g);
    std::fwrite(Li.data(), 8, p * p, g);
    std::fwrite(w.data(), 8, p, g);
    std::fwrite(gw.data(), 8, p, g);
    std::fwrite(&tr, 8, 1, g);
    std::fclose(g);
    return 0;
}
"""

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
void oracle_csr_spmm(int64_t, int64_t, const int64_t *, const int32_t *, const double *, const double *, double *);
void oracle_csr_shifted_spmm(int64_t, int64_t, const int64_t *, const int32_t *, const double *, const double *,
                         const double *, const double *, double *);
/* reads n, p, a CSR matrix pair (values a, b), lam[p], X (n x p); writes A X and (a - lam b) X */
int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "rb");
    int64_t n, p, nnz;
    if (fread(&n, 8, 1, f) != 1 || fread(&p, 8, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 2;
    int64_t *rp = malloc(8 * (n + 1));
    int32_t *col = malloc(4 * nnz);
    double *a = malloc(8 * nnz), *b = malloc(8 * nnz), *lam = malloc(8 * p), *X = malloc(8 * n * p);
    double *Y = malloc(8 * n * p), *Q = malloc(8 * n * p);
    if (fread(rp, 8, n + 1, f) != (size_t)(n + 1) || fread(col, 4, nnz, f) != (size_t)nnz ||
        fread(a, 8, nnz, f) != (size_t)nnz || fread(b, 8, nnz, f) != (size_t)nnz || fread(lam, 8, p, f) != (size_t)p ||
        fread(X, 8, n * p, f) != (size_t)(n * p)) return 2;
    fclose(f);
    oracle_csr_spmm(n, p, rp, col, a, X, Y);
    oracle_csr_shifted_spmm(n, p, rp, col, a, b, lam, X, Q);
    FILE *g = fopen(argv[2], "wb");
    fwrite(Y, 8, n * p, g);
    fwrite(Q, 8, n * p, g);
    fclose(g);
    free(rp); free(col); free(a); free(b); free(lam); free(X); free(Y); free(Q);
    return 0;
}
"""


def _build(tmp, name, src_text, cmd_head, extra):
    src = tmp / name
    src.write_text(src_text)
    exe = tmp / (name.split(".")[0])
    subprocess.run(cmd_head + SAN + [str(src)] + extra + ["-o", str(exe)], check=True)
    return exe


def _run(exe, *args):
    r = subprocess.run([str(exe)] + [str(a) for a in args], env=ENV, capture_output=True, text=True)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-2000:]
    return r


@pytest.fixture(scope="module")
def graded():
    Z = np.array([6.0, 1.0, 8.0])
    R = np.array([[0.3, -0.2, 0.1], [-1.4, 0.9, 0.4], [1.1, 1.3, -0.9]])
    mesh = wl.graded_mesh(5.0, Z, R, gamma1=0.5, gamma2=1.2, hmin=0.1)
    return fem.discretize(mesh, Z, R)


def _write_pattern(path, rp, col, hm=76, rm=16, em=64):
    with open(path, "wb") as f:
        f.write(np.int64(len(rp) - 1).tobytes())
        f.write(np.array([hm, rm, em], dtype=np.int32).tobytes())
        f.write(np.asarray(rp, dtype=np.int64).tobytes())
        f.write(np.asarray(col, dtype=np.int32).tobytes())


def test_halo_plan_under_sanitizers(tmp_path, graded):
    exe = _build(tmp_path, "halo.cpp", HALO_DRIVER, ["g++", "-std=c++17", "-I", CSRC], [])
    d = graded
    cases = [("fem", d.row_ptr, d.col, 0)]
    rng = np.random.default_rng(1)
    # random pattern with duplicate columns and empty rows
    n = 3000
    lens = rng.integers(0, 12, n)
    rp = np.concatenate([[0], np.cumsum(lens)])
    col = np.concatenate([np.sort(np.clip(i + rng.integers(-40, 40, l), 0, n - 1)) for i, l in enumerate(lens)])
    cases.append(("random", rp, col.astype(np.int32), 0))
    # malformed: a column out of range, and a row wider than the entry cap
    bad = col.astype(np.int32).copy()
    bad[len(bad) // 2] = n + 5
    cases.append(("bad index", rp, bad, 1))
    wide_rp = np.concatenate([[0, 70], 70 + np.arange(1, 80)]).astype(np.int64)      # 80 rows, row 0 has 70 entries
    wide_col = np.concatenate([np.arange(70), np.arange(1, 80)]).astype(np.int32)
    cases.append(("wide row", wide_rp, wide_col, 1))
    for name, rp_, col_, expect_fail in cases:
        inp = tmp_path / f"{name.replace(' ', '_')}.bin"
        _write_pattern(inp, rp_, col_)
        r = _run(exe, inp)
        assert r.returncode == 0, (name, r.stderr[-2000:])
        rc, rc2, nb = (int(v) for v in r.stdout.split())
        if expect_fail:
            assert rc != 0, name
        else:
            assert rc == 0 and rc2 == 0 and nb > 0, (name, rc, rc2, nb)


@pytest.mark.parametrize("p", [1, 2, 7, 33, 64, 300])
def test_dense_algebra_under_sanitizers(tmp_path, p):
    exe = _build(tmp_path, "dense.cpp", DENSE_DRIVER, ["g++", "-std=c++17", "-I", CSRC], [])
    rng = np.random.default_rng(p)
    M = rng.standard_normal((p, p))
    A = M + M.T
    Q = rng.standard_normal((p, p))
    S = Q @ Q.T + p * np.eye(p)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.int32(p).tobytes())
        f.write(A.tobytes())
        f.write(S.tobytes())
    r = _run(exe, inp, out)
    assert r.returncode == 0, r.stderr[-2000:]
    v = np.fromfile(out, dtype=np.float64)
    L, Li = v[: p * p].reshape(p, p), v[p * p: 2 * p * p].reshape(p, p)
    w, gw, tr = v[2 * p * p: 2 * p * p + p], v[2 * p * p + p: 2 * p * p + 2 * p], v[-1]
    assert np.allclose(L, np.linalg.cholesky(S), rtol=1e-12, atol=1e-12)
    assert np.allclose(Li @ L, np.eye(p), atol=1e-12)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(A), rtol=1e-10, atol=1e-10)
    assert np.allclose(np.sort(gw), sla.eigh(A, S, eigvals_only=True), rtol=1e-10, atol=1e-12)
    assert abs(tr - np.trace(np.linalg.solve(S, A))) < 1e-10 * max(1.0, abs(tr))


def test_oracle_loops_under_sanitizers(tmp_path, graded):
    src = os.path.join(ROOT, "oracle", "csrc", "oracle_kernels.c")
    exe = _build(tmp_path, "drv.c", ORACLE_DRIVER, ["gcc", "-std=c99"], [src, "-lm"])
    d = graded
    rng = np.random.default_rng(3)
    p = 5
    X = rng.standard_normal((d.n, p))
    lam = np.array([-1.0, -0.5, 0.0, 0.25, -3.0])
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([d.n, p, d.nnz], dtype=np.int64).tobytes())
        f.write(d.row_ptr.astype(np.int64).tobytes())
        f.write(d.col.astype(np.int32).tobytes())
        f.write((0.5 * d.L).tobytes())
        f.write(d.B.tobytes())
        f.write(lam.tobytes())
        f.write(X.tobytes())
    r = _run(exe, inp, out)
    assert r.returncode == 0, r.stderr[-2000:]
    v = np.fromfile(out, dtype=np.float64).reshape(2, d.n, p)
    assert np.allclose(v[0], d.csr(0.5 * d.L) @ X, rtol=1e-13, atol=1e-13)
    for l in range(p):
        ref = d.csr(0.5 * d.L - lam[l] * d.B) @ X[:, l]
        assert np.allclose(v[1][:, l], ref, rtol=1e-13, atol=1e-13)
