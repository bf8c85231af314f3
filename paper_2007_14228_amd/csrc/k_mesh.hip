// Discretization on the device (Section 2.2): interior-DOF numbering, the
// node-to-tetrahedron incidence, the sorted CSR pattern of the P1 matrices,
// element geometry, V_ext at quadrature points and the assembly of L, B and
// potential matrices M(V).
//
// Assembly is a gather: the thread that owns row i walks the tetrahedra that
// touch node i in ascending order and adds each element entry (a, b) into its
// own row.  No atomics touch values, so every sum has a fixed order.
// Incidence lists are filled with atomics (order unspecified) and then sorted
// per node, which makes the CSR pattern and all values reproducible.
#include "common.hpp"

#define OFKS_MAX_INC 128
#define OFKS_MAX_ROW 64

namespace ofks {

// 4-point degree-2 rule: barycentric (a, b, b, b) and permutations, weights |K|/4.
#define OFKS_QA 0.58541019662496845446   // (5 + 3 sqrt 5) / 20
#define OFKS_QB 0.13819660112501051518   // (5 - sqrt 5) / 20

__device__ __forceinline__ double bary(int q, int a) { return q == a ? OFKS_QA : OFKS_QB; }

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts into int64 offsets (out[n] = total)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_block(int64_t n, const int32_t *__restrict__ in,
                                                   int64_t *__restrict__ out,
                                                   int64_t *__restrict__ bsum) {
    __shared__ int64_t sh[1024];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    for (int k = threadIdx.x; k < 1024; k += 256) {
        const int64_t i = base + k;
        sh[k] = i < n ? in[i] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = sh[k];
            sh[k] = s;
            s += v;
        }
        bsum[blockIdx.x] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 1024; k += 256) {
        const int64_t i = base + k;
        if (i < n) out[i] = sh[k];
    }
}

__global__ void k_scan_bsum(int64_t nb, int64_t *__restrict__ bsum, int64_t *__restrict__ total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t s = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t v = bsum[b];
        bsum[b] = s;
        s += v;
    }
    *total = s;
}

__global__ void k_scan_add(int64_t n, int64_t *__restrict__ out, const int64_t *__restrict__ bsum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / 1024];
}

// ---------------------------------------------------------------------------
__global__ void k_interior_flags(int64_t nn, const uint8_t *__restrict__ dir, int32_t *__restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nn) f[i] = dir[i] ? 0 : 1;
}

__global__ void k_dof(int64_t nn, const uint8_t *__restrict__ dir, const int64_t *__restrict__ scan,
                      int32_t *__restrict__ dof) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nn) dof[i] = dir[i] ? -1 : (int32_t)scan[i];
}

__global__ void k_inc_count(int64_t nt, const int32_t *__restrict__ tets, int32_t *__restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nt)
        for (int a = 0; a < 4; ++a) atomicAdd(&cnt[tets[4 * t + a]], 1);
}

__global__ void k_inc_fill(int64_t nt, const int32_t *__restrict__ tets, const int64_t *__restrict__ ptr,
                           int32_t *__restrict__ cursor, int32_t *__restrict__ inc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nt)
        for (int a = 0; a < 4; ++a) {
            const int32_t v = tets[4 * t + a];
            const int32_t slot = atomicAdd(&cursor[v], 1);
            inc[ptr[v] + slot] = (int32_t)(t * 4 + a);   // tet id and local vertex
        }
}

__global__ void k_inc_sort(int64_t nn, const int64_t *__restrict__ ptr, int32_t *__restrict__ inc,
                           int32_t *__restrict__ err) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const int64_t b = ptr[v], e = ptr[v + 1];
    if (e - b > OFKS_MAX_INC) { atomicOr(err, 1); return; }
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t key = inc[i];
        int64_t j = i - 1;
        while (j >= b && inc[j] > key) { inc[j + 1] = inc[j]; --j; }
        inc[j + 1] = key;
    }
}

// Row pattern of node v: sorted unique interior DOFs of all incident tets.
// fill == 0: rowcnt[dof] = count;  fill == 1: write col[row_ptr[dof] + k].
__global__ void k_row_pattern(int64_t nn, int fill, const int32_t *__restrict__ dof,
                              const int64_t *__restrict__ iptr, const int32_t *__restrict__ inc,
                              const int32_t *__restrict__ tets, int32_t *__restrict__ rowcnt,
                              const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                              int32_t *__restrict__ err) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const int32_t i = dof[v];
    if (i < 0) return;
    int32_t cols[OFKS_MAX_ROW];
    int cnt = 0;
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
        const int64_t t = inc[k] >> 2;
        for (int b = 0; b < 4; ++b) {
            const int32_t j = dof[tets[4 * t + b]];
            if (j < 0) continue;
            int pos = 0;
            while (pos < cnt && cols[pos] < j) ++pos;
            if (pos < cnt && cols[pos] == j) continue;
            if (cnt == OFKS_MAX_ROW) { atomicOr(err, 2); return; }
            for (int q = cnt; q > pos; --q) cols[q] = cols[q - 1];
            cols[pos] = j;
            ++cnt;
        }
    }
    if (!fill) {
        rowcnt[i] = cnt;
    } else {
        const int64_t o = row_ptr[i];
        for (int q = 0; q < cnt; ++q) col[o + q] = cols[q];
    }
}

// geom[13 t + 0] = |K|, geom[13 t + 1 + 3 a + d] = d lambda_a / d x_d
__global__ void k_tet_geom(int64_t nt, const double *__restrict__ xyz, const int32_t *__restrict__ tets,
                           double *__restrict__ geom, int32_t *__restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double v[4][3];
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) v[a][d] = xyz[3 * (int64_t)tets[4 * t + a] + d];
    double e1[3], e2[3], e3[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = v[1][d] - v[0][d];
        e2[d] = v[2][d] - v[0][d];
        e3[d] = v[3][d] - v[0][d];
    }
    const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
    const double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
    const double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
    if (!(fabs(det) > 0.0)) atomicOr(err, 4);
    double *g = geom + 13 * t;
    g[0] = fabs(det) / 6.0;
    for (int d = 0; d < 3; ++d) {
        const double g1 = c23[d] / det, g2 = c31[d] / det, g3 = c12[d] / det;
        g[1 + 3 + d] = g1;
        g[1 + 6 + d] = g2;
        g[1 + 9 + d] = g3;
        g[1 + d] = -(g1 + g2 + g3);
    }
}

// V_ext(r) = -sum_j Z_j / |r - R_j| at the 4 quadrature points (eq. ext)
__global__ void k_vext(int64_t nt, const double *__restrict__ xyz, const int32_t *__restrict__ tets, int M,
                       const double *__restrict__ Z, const double *__restrict__ R, double *__restrict__ vq) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double v[4][3];
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) v[a][d] = xyz[3 * (int64_t)tets[4 * t + a] + d];
    for (int q = 0; q < 4; ++q) {
        double x[3];
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int a = 0; a < 4; ++a) s += bary(q, a) * v[a][d];
            x[d] = s;
        }
        double V = 0.0;
        for (int j = 0; j < M; ++j) {
            const double dx = x[0] - R[3 * j], dy = x[1] - R[3 * j + 1], dz = x[2] - R[3 * j + 2];
            V -= Z[j] / sqrt(dx * dx + dy * dy + dz * dz);
        }
        vq[4 * t + q] = V;
    }
}

// Row-gather assembly.  mode 0: L, B, M(vq) and the interleaved pairs
// hb = (L/2 + M, B), lb = (L/2, B), plus the diagonals.  mode 1: hb.x and
// hdiag only (H = L/2 + M(vq) with L from Lv).
__global__ __launch_bounds__(128) void k_assemble(int64_t nn, int mode, const int32_t *__restrict__ dof,
                                                 const int64_t *__restrict__ iptr,
                                                 const int32_t *__restrict__ inc,
                                                 const int32_t *__restrict__ tets,
                                                 const double *__restrict__ geom,
                                                 const double *__restrict__ vq,
                                                 const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col, double *__restrict__ Lv,
                                                 double *__restrict__ Bv, double *__restrict__ Mv,
                                                 double2 *__restrict__ hb, double2 *__restrict__ lb,
                                                 double *__restrict__ lhd, double *__restrict__ bd,
                                                 double *__restrict__ hd) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    const int32_t i = dof[v];
    if (i < 0) return;
    const int64_t r0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - r0);
    double lacc[OFKS_MAX_ROW], bacc[OFKS_MAX_ROW], macc[OFKS_MAX_ROW];
    for (int k = 0; k < len; ++k) { lacc[k] = 0.0; bacc[k] = 0.0; macc[k] = 0.0; }
    for (int64_t k = iptr[v]; k < iptr[v + 1]; ++k) {
        const int64_t t = inc[k] >> 2;
        const int a = inc[k] & 3;
        const double *g = geom + 13 * t;
        const double vol = g[0];
        double w[4];
        for (int q = 0; q < 4; ++q) w[q] = 0.25 * vol * vq[4 * t + q];
        for (int b = 0; b < 4; ++b) {
            const int32_t j = dof[tets[4 * t + b]];
            if (j < 0) continue;
            int pos = 0;
            while (pos < len && col[r0 + pos] != j) ++pos;
            if (pos == len) continue;   // cannot happen: the pattern came from the same incidence
            double m = 0.0;
            for (int q = 0; q < 4; ++q) m += w[q] * bary(q, a) * bary(q, b);
            macc[pos] += m;
            if (mode == 0) {
                lacc[pos] += vol * (g[1 + 3 * a] * g[1 + 3 * b] + g[2 + 3 * a] * g[2 + 3 * b] +
                                    g[3 + 3 * a] * g[3 + 3 * b]);
                bacc[pos] += vol * (a == b ? 2.0 : 1.0) / 20.0;
            }
        }
    }
    for (int k = 0; k < len; ++k) {
        const int64_t e = r0 + k;
        const bool diag = col[e] == i;
        if (mode == 0) {
            Lv[e] = lacc[k];
            Bv[e] = bacc[k];
            Mv[e] = macc[k];
            hb[e] = make_double2(0.5 * lacc[k] + macc[k], bacc[k]);
            lb[e] = make_double2(0.5 * lacc[k], bacc[k]);
            if (diag) { lhd[i] = 0.5 * lacc[k]; bd[i] = bacc[k]; hd[i] = 0.5 * lacc[k] + macc[k]; }
        } else {
            const double h = 0.5 * Lv[e] + macc[k];
            hb[e].x = h;
            if (diag) hd[i] = h;
        }
    }
}

__global__ void k_pairs_to_f32(int64_t m, const double2 *__restrict__ a, float2 *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void k_split_pairs(int64_t m, const double2 *__restrict__ a, double *__restrict__ x,
                              double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = a[i].x;
        y[i] = a[i].y;
    }
}

__global__ void k_make_pairs(int64_t m, const double *__restrict__ x, const double *__restrict__ y,
                             double2 *__restrict__ a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = make_double2(x[i], y[i]);
}

// diagonal values of CSR arrays (pattern has the diagonal in every row)
__global__ void k_diag(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                       const double2 *__restrict__ pairs, double *__restrict__ dx, double *__restrict__ dy,
                       int32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
        if (col[e] == i) {
            if (dx) dx[i] = pairs[e].x;
            if (dy) dy[i] = pairs[e].y;
            return;
        }
    atomicOr(err, 8);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t scan_exclusive(hipStream_t s, int64_t n, const int32_t *in, int64_t *out, int64_t *bsum) {
    const int64_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, s, n, in, out, bsum);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1), 0, s, nb, bsum, out + n);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n, 256)), dim3(256), 0, s, n, out, bsum);
    return hipGetLastError();
}

hipError_t launch_interior_flags(hipStream_t s, int64_t nn, const uint8_t *dir, int32_t *f) {
    hipLaunchKernelGGL(k_interior_flags, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, dir, f);
    return hipGetLastError();
}
hipError_t launch_dof(hipStream_t s, int64_t nn, const uint8_t *dir, const int64_t *scan, int32_t *dof) {
    hipLaunchKernelGGL(k_dof, dim3(nblk(nn, 256)), dim3(256), 0, s, nn, dir, scan, dof);
    return hipGetLastError();
}
hipError_t launch_inc_count(hipStream_t s, int64_t nt, const int32_t *tets, int32_t *cnt) {
    hipLaunchKernelGGL(k_inc_count, dim3(nblk(nt, 256)), dim3(256), 0, s, nt, tets, cnt);
    return hipGetLastError();
}
hipError_t launch_inc_fill(hipStream_t s, int64_t nt, const int32_t *tets, const int64_t *ptr, int32_t *cursor,
                           int32_t *inc) {
    hipLaunchKernelGGL(k_inc_fill, dim3(nblk(nt, 256)), dim3(256), 0, s, nt, tets, ptr, cursor, inc);
    return hipGetLastError();
}
hipError_t launch_inc_sort(hipStream_t s, int64_t nn, const int64_t *ptr, int32_t *inc, int32_t *err) {
    hipLaunchKernelGGL(k_inc_sort, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, ptr, inc, err);
    return hipGetLastError();
}
hipError_t launch_row_pattern(hipStream_t s, int64_t nn, int fill, const int32_t *dof, const int64_t *iptr,
                              const int32_t *inc, const int32_t *tets, int32_t *rowcnt, const int64_t *rp,
                              int32_t *col, int32_t *err) {
    hipLaunchKernelGGL(k_row_pattern, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, fill, dof, iptr, inc, tets,
                       rowcnt, rp, col, err);
    return hipGetLastError();
}
hipError_t launch_tet_geom(hipStream_t s, int64_t nt, const double *xyz, const int32_t *tets, double *geom,
                           int32_t *err) {
    hipLaunchKernelGGL(k_tet_geom, dim3(nblk(nt, 256)), dim3(256), 0, s, nt, xyz, tets, geom, err);
    return hipGetLastError();
}
hipError_t launch_vext(hipStream_t s, int64_t nt, const double *xyz, const int32_t *tets, int M, const double *Z,
                       const double *R, double *vq) {
    hipLaunchKernelGGL(k_vext, dim3(nblk(nt, 256)), dim3(256), 0, s, nt, xyz, tets, M, Z, R, vq);
    return hipGetLastError();
}
hipError_t launch_assemble(hipStream_t s, int64_t nn, int mode, const int32_t *dof, const int64_t *iptr,
                           const int32_t *inc, const int32_t *tets, const double *geom, const double *vq,
                           const int64_t *rp, const int32_t *col, double *Lv, double *Bv, double *Mv,
                           double2 *hb, double2 *lb, double *lhd, double *bd, double *hd) {
    hipLaunchKernelGGL(k_assemble, dim3(nblk(nn, 128)), dim3(128), 0, s, nn, mode, dof, iptr, inc, tets, geom,
                       vq, rp, col, Lv, Bv, Mv, hb, lb, lhd, bd, hd);
    return hipGetLastError();
}
hipError_t launch_pairs_to_f32(hipStream_t s, int64_t m, const double2 *a, float2 *b) {
    hipLaunchKernelGGL(k_pairs_to_f32, dim3(2048), dim3(256), 0, s, m, a, b);
    return hipGetLastError();
}
hipError_t launch_split_pairs(hipStream_t s, int64_t m, const double2 *a, double *x, double *y) {
    hipLaunchKernelGGL(k_split_pairs, dim3(2048), dim3(256), 0, s, m, a, x, y);
    return hipGetLastError();
}
hipError_t launch_make_pairs(hipStream_t s, int64_t m, const double *x, const double *y, double2 *a) {
    hipLaunchKernelGGL(k_make_pairs, dim3(2048), dim3(256), 0, s, m, x, y, a);
    return hipGetLastError();
}
hipError_t launch_diag(hipStream_t s, int64_t n, const int64_t *rp, const int32_t *col, const double2 *pairs,
                       double *dx, double *dy, int32_t *err) {
    hipLaunchKernelGGL(k_diag, dim3(nblk(n, 256)), dim3(256), 0, s, n, rp, col, pairs, dx, dy, err);
    return hipGetLastError();
}

}  // namespace ofks
