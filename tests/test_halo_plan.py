"""Host logic of the LDS-halo SpMM: the row-block plan (csrc/halo_plan.hpp),
compiled here with g++ and checked from outside on real and adversarial CSR
patterns.  What the plan must satisfy: every row in exactly one block of
consecutive rows, at most rmax rows per block, the halo sorted and equal to
the block's columns together with its rows (at most hmax), the rows at
consecutive slots from rbase, every entry's slot pointing back to its own
column, and greedy blocks (the next row would not have fit)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as wl
from oracle import fem

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2007_14228_amd", "csrc", "halo_plan.hpp")

DRIVER = r"""
#include "halo_plan.hpp"
#include <cstdio>
#include <vector>
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
    FILE *g = std::fopen(argv[2], "wb");
    int64_t nb = P.nb(), hl = (int64_t)P.halo.size(), nl = (int64_t)P.lcol.size();
    std::fwrite(&rc, 4, 1, g); std::fwrite(&rc2, 4, 1, g); std::fwrite(&where, 8, 1, g);
    std::fwrite(&nb, 8, 1, g); std::fwrite(&hl, 8, 1, g); std::fwrite(&nl, 8, 1, g);
    std::fwrite(P.row0.data(), 8, P.row0.size(), g); std::fwrite(P.hoff.data(), 8, P.hoff.size(), g);
    std::fwrite(P.halo.data(), 4, hl, g); std::fwrite(P.lcol.data(), 2, nl, g);
    std::fwrite(P.rbase.data(), 4, P.rbase.size(), g);
    std::fclose(g);
    return 0;
}
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("halo")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)], check=True)

    def run(rp, col, hmax=160, rmax=64, emax=64):
        rp = np.asarray(rp, np.int64)
        col = np.asarray(col, np.int32)
        inp, out = d / "in.bin", d / "out.bin"
        with open(inp, "wb") as f:
            f.write(np.int64(len(rp) - 1).tobytes() + np.int32(hmax).tobytes() + np.int32(rmax).tobytes() +
                    np.int32(emax).tobytes())
            f.write(rp.tobytes() + col.tobytes())
        subprocess.run([str(exe), str(inp), str(out)], check=True)
        b = open(out, "rb").read()
        rc, rc2 = np.frombuffer(b[:8], np.int32)
        where, nb, hl, nl = np.frombuffer(b[8:40], np.int64)
        o = 40
        row0 = np.frombuffer(b[o:o + 8 * (nb + 1)], np.int64); o += 8 * (nb + 1)
        hoff = np.frombuffer(b[o:o + 8 * (nb + 1)], np.int64); o += 8 * (nb + 1)
        halo = np.frombuffer(b[o:o + 4 * hl], np.int32); o += 4 * hl
        lcol = np.frombuffer(b[o:o + 2 * nl], np.uint16); o += 2 * nl
        rbase = np.frombuffer(b[o:o + 4 * nb], np.int32)
        return dict(rc=int(rc), rc2=int(rc2), where=int(where), nb=int(nb), row0=row0, hoff=hoff, halo=halo,
                    lcol=lcol, rbase=rbase)
    return run


def _check_plan(P, rp, col, hmax, rmax, emax=64):
    n = len(rp) - 1
    assert P["rc"] == 0 and P["rc2"] == 0
    assert np.diff(rp).max() <= emax
    row0, hoff, halo, lcol, rbase = P["row0"], P["hoff"], P["halo"], P["lcol"], P["rbase"]
    assert row0[0] == 0 and row0[-1] == n and np.all(np.diff(row0) >= 1) and np.all(np.diff(row0) <= rmax)
    assert hoff[0] == 0 and hoff[-1] == len(halo)
    for b in range(P["nb"]):
        r0, r1 = row0[b], row0[b + 1]
        cols = col[rp[r0]:rp[r1]]
        h = halo[hoff[b]:hoff[b + 1]]
        assert np.array_equal(h, np.union1d(cols, np.arange(r0, r1)))   # sorted: the columns and the rows
        assert len(h) <= hmax
        assert np.array_equal(h[lcol[rp[r0]:rp[r1]]], cols)    # every slot maps back
        assert np.array_equal(h[rbase[b]:rbase[b] + (r1 - r0)], np.arange(r0, r1))
        if r1 < n:                                             # greedy: the next row would not fit
            nxt = np.union1d(h, np.append(col[rp[r1]:rp[r1 + 1]], r1))
            assert r1 - r0 == rmax or len(nxt) > hmax


def test_plan_on_fem_pattern(planner):
    w = wl.make_workload("c1")
    d = fem.discretize(w.mesh, w.Z, w.R)
    for hmax, rmax in [(160, 64), (40, 64), (160, 7), (64, 1)]:
        P = planner(d.row_ptr, d.col, hmax, rmax)
        _check_plan(P, d.row_ptr, d.col, hmax, rmax)
    P = planner(d.row_ptr, d.col)
    # on a tetrahedral mesh the halo is a few times the row count, far below nnz
    rows = np.diff(P["row0"])
    hal = np.diff(P["hoff"])
    assert hal.sum() < 0.5 * d.nnz and rows.mean() > 8
    # every FEM row has its diagonal: adding the rows changes no halo
    for b in range(P["nb"]):
        r0, r1 = P["row0"][b], P["row0"][b + 1]
        assert hal[b] == len(np.unique(d.col[d.row_ptr[r0]:d.row_ptr[r1]]))


def test_plan_on_random_patterns(planner):
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(1, 400))
        lens = rng.integers(0, 30, n)
        rp = np.concatenate([[0], np.cumsum(lens)])
        col = rng.integers(0, n, rp[-1]).astype(np.int32)   # duplicates and empty rows included
        hmax, rmax = int(rng.integers(30, 200)), int(rng.integers(1, 70))
        P = planner(rp, col, hmax, rmax)
        _check_plan(P, rp, col, hmax, rmax)


def test_plan_with_empty_rows(planner):
    # 100 empty rows first (blocks whose halo is just their rows), then a band matrix
    n = 400
    lens = np.concatenate([np.zeros(100, np.int64), np.full(n - 100, 3)])
    rp = np.concatenate([[0], np.cumsum(lens)])
    col = np.concatenate([[max(r - 1, 100), r, min(r + 1, n - 1)] for r in range(100, n)]).astype(np.int32)
    P = planner(rp, col)
    _check_plan(P, rp, col, 160, 64)
    assert P["hoff"][1] == 64 and P["rbase"][0] == 0   # rows 0..63: the halo is the rows


def test_plan_refuses_too_wide_rows_and_bad_indices(planner):
    n = 300
    rp = np.array([0, 3, 3 + 200] + [203 + k for k in range(1, n - 1)], np.int64)
    col = np.concatenate([[0, 1, 2], np.arange(200), np.arange(2, n)]).astype(np.int32)
    assert len(col) == rp[-1]
    P = planner(rp, col, hmax=160, emax=256)
    assert P["rc"] == 1 and P["where"] == 1 and P["nb"] == 0        # row 1 alone has 200 columns
    assert planner(rp, col, hmax=200, emax=256)["rc"] == 0
    P = planner(rp, col, hmax=200, emax=64)                           # ... and 200 entries
    assert P["rc"] == 1 and P["where"] == 1
    bad = col.copy()
    bad[5] = n
    P = planner(rp, bad, hmax=200, emax=256)
    assert P["rc"] == -2 and P["where"] == 5
    bad[5] = -1
    assert planner(rp, bad, hmax=200, emax=256)["rc"] == -2
    rp2 = rp.copy()
    rp2[4] = rp2[3] - 1
    assert planner(rp2, col, hmax=200, emax=256)["rc"] == -1
