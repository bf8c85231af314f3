// Host-side plan of the LDS-halo SpMM (k_spmm_halo): consecutive CSR rows, each
// with at most emax entries, are grouped greedily into blocks of at most rmax
// rows whose halo (the distinct columns of the rows together with the rows
// themselves, kept sorted) numbers at most hmax entries.  The block's rows
// then sit at consecutive halo slots from rbase[b]; lcol[e] is the slot of
// entry e's column in its block's halo.  Plain C++ (no HIP), so the host
// tests compile it with g++.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace ofks {

struct HaloPlan {
    std::vector<int64_t> row0{0};   // block b owns rows [row0[b], row0[b+1])
    std::vector<int64_t> hoff{0};   // block b's halo is halo[hoff[b] .. hoff[b+1])
    std::vector<int32_t> halo;      // ascending within a block
    std::vector<uint16_t> lcol;     // per CSR entry
    std::vector<int32_t> rbase;     // halo slot of block b's first row
    int64_t nb() const { return (int64_t)row0.size() - 1; }
};

enum { HALO_OK = 0, HALO_TOO_WIDE = 1, HALO_BAD_ROWPTR = -1, HALO_BAD_COLUMN = -2, HALO_BAD_PLAN = -3 };

// Build the plan.  HALO_TOO_WIDE: some row has more than emax entries or
// alone a halo of more than hmax (no plan); HALO_BAD_*: the CSR arrays
// are malformed (*where = row or entry).  hmax <= 65536 so that a slot fits in
// 16 bits.
inline int halo_plan_build(int64_t n, const int64_t *rp, const int32_t *col, int hmax, int rmax, int emax,
                           HaloPlan &P, int64_t *where) {
    P = HaloPlan();
    if (n <= 0 || rp[0] != 0) { *where = 0; return HALO_BAD_ROWPTR; }
    const int64_t nnz = rp[n];
    if (hmax < 1 || hmax > 65536 || rmax < 1) { *where = 0; return HALO_BAD_PLAN; }
    std::vector<int64_t> stamp(n, -1);   // b: in block b's halo; -(b + 2): counted for block b, not yet added
    std::vector<int32_t> slot(n, 0);
    std::vector<int32_t> cur;
    P.lcol.assign((size_t)std::max<int64_t>(nnz, 0), 0);
    P.halo.reserve((size_t)(3.5 * n) + 64);
    int64_t b = 0, start = 0;
    auto close = [&](int64_t end) {
        std::sort(cur.begin(), cur.end());
        for (size_t k = 0; k < cur.size(); ++k) slot[cur[k]] = (int32_t)k;
        for (int64_t e = rp[start]; e < rp[end]; ++e) P.lcol[e] = (uint16_t)slot[col[e]];
        P.rbase.push_back(slot[start]);
        P.halo.insert(P.halo.end(), cur.begin(), cur.end());
        P.row0.push_back(end);
        P.hoff.push_back((int64_t)P.halo.size());
        cur.clear();
        ++b;
        start = end;
    };
    for (int64_t r = 0; r < n; ++r) {
        if (rp[r + 1] < rp[r] || rp[r + 1] > nnz) { *where = r; return HALO_BAD_ROWPTR; }
        if (rp[r + 1] - rp[r] > emax) { *where = r; P = HaloPlan(); return HALO_TOO_WIDE; }
        for (int pass = 0;; ++pass) {
            int64_t fresh = 0;
            for (int64_t e = rp[r]; e <= rp[r + 1]; ++e) {   // the entries, then the row itself
                const int64_t cc = e < rp[r + 1] ? col[e] : r;
                if (cc < 0 || cc >= n) { *where = e; return HALO_BAD_COLUMN; }
                if (stamp[cc] != b && stamp[cc] != -(b + 2)) {
                    stamp[cc] = -(b + 2);
                    ++fresh;
                }
            }
            if ((int64_t)cur.size() + fresh <= hmax && r - start < rmax) break;
            if (pass == 1 || r == start) { *where = r; P = HaloPlan(); return HALO_TOO_WIDE; }
            close(r);   // the row opens the next block; count it again there
        }
        for (int64_t e = rp[r]; e <= rp[r + 1]; ++e) {
            const int32_t cc = e < rp[r + 1] ? col[e] : (int32_t)r;
            if (stamp[cc] != b) {
                stamp[cc] = b;
                cur.push_back(cc);
            }
        }
    }
    close(n);
    return HALO_OK;
}

// Independent check of a plan against the CSR arrays: every row covered once,
// block and row sizes within bounds, every slot in range and mapping back to
// its column, the block's rows at slots rbase[b] + (r - row0[b]).
inline int halo_plan_check(int64_t n, const int64_t *rp, const int32_t *col, int hmax, int rmax, int emax,
                           const HaloPlan &P, int64_t *where) {
    const int64_t nb = P.nb();
    if (nb < 1 || P.row0[0] != 0 || P.row0[nb] != n || (int64_t)P.hoff.size() != nb + 1 || P.hoff[0] != 0 ||
        P.hoff[nb] != (int64_t)P.halo.size() || (int64_t)P.lcol.size() != rp[n] || (int64_t)P.rbase.size() != nb) {
        *where = -1;
        return HALO_BAD_PLAN;
    }
    for (int64_t k = 0; k < nb; ++k) {
        const int64_t hn = P.hoff[k + 1] - P.hoff[k];
        if (P.row0[k + 1] <= P.row0[k] || P.row0[k + 1] - P.row0[k] > rmax || hn < P.row0[k + 1] - P.row0[k] ||
            hn > hmax || P.rbase[k] < 0 || P.rbase[k] + (P.row0[k + 1] - P.row0[k]) > hn) {
            *where = k;
            return HALO_BAD_PLAN;
        }
        for (int64_t r = P.row0[k]; r < P.row0[k + 1]; ++r)
            if (P.halo[P.hoff[k] + P.rbase[k] + (r - P.row0[k])] != r) {
                *where = r;
                return HALO_BAD_PLAN;
            }
        for (int64_t r = P.row0[k]; r < P.row0[k + 1]; ++r)
            if (rp[r + 1] - rp[r] > emax) {
                *where = r;
                return HALO_BAD_PLAN;
            }
        for (int64_t e = rp[P.row0[k]]; e < rp[P.row0[k + 1]]; ++e)
            if (P.lcol[e] >= hn || P.halo[P.hoff[k] + P.lcol[e]] != col[e]) {
                *where = e;
                return HALO_BAD_PLAN;
            }
    }
    return HALO_OK;
}

}  // namespace ofks
